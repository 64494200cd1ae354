// scc.hip -- decomposition into strongly connected components on gfx950 by
// forward-backward search with trimming (Section 1.1: trimming removes the
// size-1 components cheaply, before and after FW-BW takes out the large one).
//
// Phases, driven from the host (each ends with a few counters read back):
//  1. Two-sided AC-6 trimming (ac6_two.hip) with the vertices already
//     assigned preset as removed.  A vertex it removes lies on no cycle of
//     the unassigned vertices, so it is a component of its own.
//  2. Forward-backward search from one pivot, the unassigned vertex with the
//     largest (outdeg + 1)(indeg + 1): the vertices that the pivot reaches
//     and that reach the pivot form its component (the large one on
//     power-law graphs).
//  3. Trimming again.
//  4. Colouring rounds while unassigned vertices remain: every unassigned
//     vertex takes the largest id among the unassigned vertices that reach it
//     (max-label propagation over edges between unassigned vertices).  A
//     vertex r that keeps its own id is a root; every vertex of colour r is
//     reached from r, so the vertices of colour r that reach r (a backward
//     search inside the colour) are exactly r's component.  The largest
//     unassigned id is always a root, so every round assigns at least one
//     component.  Then trimming again.
// Between 3 and 4, the size-2 check: two unassigned vertices that are each
// other's only unassigned predecessor (or only unassigned successor) form a
// component of two, labelled with the smaller id; trimming follows if any
// were found.
// label[v] is the id of one vertex of v's component (v itself, the pivot,
// the pair's smaller id or the root); equal labels mean one component.
//
// The searches go level by level over a frontier of items (a vertex and a
// direction: forward follows successors, backward predecessors).  A level
// scans the frontier's list lengths, then deals their entries out evenly: each
// block takes a contiguous range of kLBS entries, stages the frontier items
// that own them in LDS and finds each entry's owner by binary search, so a hub
// and a thousand short lists cost the same per entry.  A neighbour is taken
// once per direction, by the lane whose fetch-or sets its mark first, and
// appended to the next frontier.
#include <chrono>

#include "trim_device.h"
#include "trim_internal.h"
#include "scc_internal.h"

namespace trim {

namespace {

__device__ __forceinline__ bool has_bit(const uint32_t* bm, int v) {
    return (bm[v >> 5] >> (v & 31)) & 1u;
}
__device__ __forceinline__ int or_dev(int* p, int v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int max_dev(int* p, int v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_misc(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long block_total(unsigned long long x,
                                                          unsigned long long* red) {
    return block_sum((uint64_t)x, reinterpret_cast<uint64_t*>(red));
}

__global__ void scc_init(int n, int* label, int* flags, uint32_t* assigned,
                         unsigned long long* misc) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    const int words = ((n + 31) >> 5) + 2;
    for (int v = tid; v < n; v += stride) {
        label[v] = -1;
        flags[v] = 0;
    }
    for (int i = tid; i < words; i += stride) assigned[i] = 0;
    if (tid < kSccMisc) misc[tid] = 0;
}

// Zeroes the misc words selected by `mask` and the queue counters, if given
// (one block).
__global__ void scc_reset(unsigned long long* misc, int mask, int* ctr) {
    if (ctr)
        for (int i = threadIdx.x; i < kCtrInts; i += blockDim.x) ctr[i] = 0;
    if (threadIdx.x < kSccMisc && ((mask >> threadIdx.x) & 1)) misc[threadIdx.x] = 0;
}

// After a trim: vertices not live and not yet assigned are components of
// their own.  assigned = not live; counts live (unassigned) vertices and the
// newly taken ones.  One thread per bitmap word.
__global__ void scc_take_trimmed(int n, const uint32_t* live, uint32_t* assigned, int* label,
                                 unsigned long long* misc) {
    __shared__ unsigned long long red[16];
    const int words = (n + 31) >> 5;
    unsigned long long active = 0, taken = 0;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < words; w += gridDim.x * blockDim.x) {
        const uint32_t valid = (w == words - 1 && (n & 31)) ? ((1u << (n & 31)) - 1u) : ~0u;
        const uint32_t lv = live[w] & valid;
        uint32_t fresh = ~lv & ~assigned[w] & valid;
        taken += (unsigned long long)__popc(fresh);
        while (fresh) {
            const int b = __ffs(fresh) - 1;
            label[w * 32 + b] = w * 32 + b;
            fresh &= fresh - 1;
        }
        assigned[w] = ~lv & valid;
        active += (unsigned long long)__popc(lv);
    }
    active = block_total(active, red);
    taken = block_total(taken, red);
    if (threadIdx.x == 0) {
        if (active) add_misc(misc + kSccActive, active);
        if (taken) add_misc(misc + kSccTaken, taken);
    }
}

// The unassigned vertex with the largest (outdeg + 1)(indeg + 1), ties to the
// larger id: misc[kSccPivot] = product << 32 | id.
__global__ void scc_pivot(int n, const int* row_off, const int* rrow_off, const uint32_t* live,
                          unsigned long long* misc) {
    unsigned long long best = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        if (!has_bit(live, v)) continue;
        const unsigned long long d = (unsigned long long)(row_off[v + 1] - row_off[v]) + 1;
        const unsigned long long di = (unsigned long long)(rrow_off[v + 1] - rrow_off[v]) + 1;
        unsigned long long p = d * di;
        if (p > 0x7FFFFFFFull) p = 0x7FFFFFFFull;
        const unsigned long long key = (p << 32) | (unsigned)v;
        best = key > best ? key : best;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned lo = __shfl_xor((unsigned)best, off);
        const unsigned hi = __shfl_xor((unsigned)(best >> 32), off);
        const unsigned long long o = ((unsigned long long)hi << 32) | lo;
        best = o > best ? o : best;
    }
    if (lane_id() == 0 && best)
        __hip_atomic_fetch_max(misc + kSccPivot, best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Search items: bit 30 = backward, low 30 bits = vertex.
__device__ __forceinline__ uint32_t ritem(int dir, int v) { return ((uint32_t)dir << 30) | (uint32_t)v; }

// The pivot, marked and placed in the frontier in both directions (one
// thread; misc[kSccFront] = 2).
__global__ void scc_seed_pivot(unsigned long long* misc, int* flags, uint32_t* front) {
    if (threadIdx.x == 0) {
        const int v = (int)(misc[kSccPivot] & 0xFFFFFFFFull);
        flags[v] = 3;
        front[0] = ritem(0, v);
        front[1] = ritem(1, v);
        misc[kSccFront] = 2;
    }
}

// Unassigned vertices: colour = own id, marks cleared.
__global__ void scc_color_init(int n, const uint32_t* live, int* color, int* flags) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        if (!has_bit(live, v)) continue;
        color[v] = v;
        flags[v] = 0;
    }
}

// One max-label sweep over the edges between unassigned vertices; sets
// misc[kSccChanged] when some colour grew.  Colours only grow, and a grown
// colour read by a later lane of the same sweep only speeds convergence.
__global__ void scc_color_sweep(int n, const int* row_off, const int* col, const uint32_t* live,
                                int* color, unsigned long long* misc) {
    bool changed = false;
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        if (!has_bit(live, u)) continue;
        const int c = ld_dev(color + u);
        const int b = row_off[u], e = row_off[u + 1];
        for (int p = b; p < e; ++p) {
            const int w = col[p];
            if (!has_bit(live, w) || ld_cached(color + w) >= c) continue;
            if (max_dev(color + w, c) < c) changed = true;
        }
    }
    if (ballot(changed) && lane_id() == 0) add_misc(misc + kSccChanged, 1);
}

// Appends this lane's item (if any) to `out` with one counter update per
// wavefront.
__device__ __forceinline__ void append_item(bool has, uint32_t it, uint32_t* out,
                                            unsigned long long* count) {
    const uint64_t m = ballot(has);
    if (!m) return;
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader)
        base = __hip_atomic_fetch_add(count, (unsigned long long)popc(m), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    base = ((unsigned long long)__shfl((unsigned)(base >> 32), leader) << 32) |
           __shfl((unsigned)base, leader);
    if (has) out[base + popc(m & lanes_below())] = it;
}

// Roots (unassigned v with colour v): marked backward, placed in the frontier
// backward (misc[kSccFront] zeroed before).
__global__ void scc_seed_roots(int n, const uint32_t* live, const int* color, int* flags,
                               uint32_t* front, unsigned long long* misc) {
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int v = base + threadIdx.x;
        const bool root = v < n && has_bit(live, v) && color[v] == v;
        if (root) flags[v] = 2;
        append_item(root, ritem(1, v), front, misc + kSccFront);
    }
}

// Takes w for direction bit `bit` if it is unassigned, in colour c (when
// colours are used) and not yet marked: the fetch-or that sets the mark wins.
__device__ __forceinline__ bool take(int w, int bit, int c, const uint32_t* live, const int* color,
                                     int* flags, bool& tried) {
    tried = false;
    if (!has_bit(live, w)) return false;
    if (color && color[w] != c) return false;
    if (ld_cached(flags + w) & bit) return false;
    tried = true;
    return (or_dev(flags + w, bit) & bit) == 0;
}

__device__ __forceinline__ uint32_t item_len(uint32_t it, const int* row_off, const int* rrow_off) {
    const int v = (int)(it & kIdMask);
    const int* off = (it >> 30) ? rrow_off : row_off;
    return (uint32_t)(off[v + 1] - off[v]);
}

// Prefix scan of the frontier's list lengths, step 1: an exclusive scan inside
// each chunk of kScanChunk items (one block of 256 threads, 4 items each);
// the chunk's total goes to bsum.
__global__ __launch_bounds__(256) void scc_scan_chunks(const uint32_t* front, const int* row_off,
                                                       const int* rrow_off, uint32_t* pre,
                                                       uint32_t* bsum,
                                                       const unsigned long long* misc) {
    __shared__ uint32_t s_w[256 / kWave];
    const long long F = (long long)misc[kSccFront];
    const long long chunks = (F + kScanChunk - 1) / kScanChunk;
    for (long long c = blockIdx.x; c < chunks; c += gridDim.x) {
        const long long i0 = c * kScanChunk + threadIdx.x * 4;
        uint32_t len[4], sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            len[j] = i0 + j < F ? item_len(front[i0 + j], row_off, rrow_off) : 0;
            sum += len[j];
        }
        // exclusive scan of the per-thread sums over the block
        uint32_t inc = sum;
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t t = __shfl_up(inc, d);
            if (lane_id() >= d) inc += t;
        }
        if (lane_id() == kWave - 1) s_w[threadIdx.x / kWave] = inc;
        __syncthreads();
        uint32_t wbase = 0;
        for (int w = 0; w < threadIdx.x / kWave; ++w) wbase += s_w[w];
        uint32_t run = wbase + inc - sum;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < F) pre[i0 + j] = run;
            run += len[j];
        }
        if (threadIdx.x == blockDim.x - 1) bsum[c] = wbase + inc;
        __syncthreads();
    }
}

// Step 2 (one block): exclusive scan of the chunk sums, and the frontier's
// total entries into misc[kSccTotal].
__global__ void scc_scan_sums(uint32_t* bsum, unsigned long long* misc) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const long long F = (long long)misc[kSccFront];
    const long long chunks = (F + kScanChunk - 1) / kScanChunk;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (long long c0 = 0; c0 < chunks; c0 += blockDim.x) {
        const long long c = c0 + threadIdx.x;
        const uint32_t x = c < chunks ? bsum[c] : 0;
        uint32_t inc = x;
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t t = __shfl_up(inc, d);
            if (lane_id() >= d) inc += t;
        }
        if (lane_id() == kWave - 1) s_w[threadIdx.x / kWave] = inc;
        __syncthreads();
        uint32_t wbase = s_carry;
        for (int w = 0; w < (int)(threadIdx.x / kWave); ++w) wbase += s_w[w];
        if (c < chunks) bsum[c] = wbase + inc - x;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) s_carry = wbase + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        misc[kSccTotal] = s_carry;
        misc[kSccEdges] += s_carry;
        misc[kSccNext] = 0;
    }
}

// Step 3: add the chunk offsets.
__global__ void scc_scan_add(uint32_t* pre, const uint32_t* bsum, const unsigned long long* misc) {
    const long long F = (long long)misc[kSccFront];
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < F;
         i += (long long)gridDim.x * blockDim.x)
        pre[i] += bsum[i / kScanChunk];
}

constexpr int kLBS = 2048;   // entries per block range of one level (256 threads x 8)

// The last index i in [0, F) with pre[i] <= key, found by the whole block: a
// 256-way search, one parallel probe round per step (three steps cover 2^24
// items) instead of a chain of dependent loads.
__device__ long long owner_search(const uint32_t* pre, long long F, unsigned long long key) {
    long long lo = 0, hi = F - 1;
    while (lo < hi) {   // block-uniform
        // step 1 probes every index of the range, so the loop ends exactly
        const long long step = (hi - lo + 1 + blockDim.x - 1) / blockDim.x;
        const long long i = lo + (long long)threadIdx.x * step;
        const bool ok = i <= hi && (unsigned long long)pre[i] <= key;
        // the probes are in order and pre[lo] <= key, so the true ones form a prefix
        const long long t = __syncthreads_count(ok);
        const long long nlo = lo + (t - 1) * step;
        const long long nhi = min(hi, lo + t * step - 1);
        lo = nlo;
        hi = step == 1 ? nlo : nhi;
    }
    return lo;
}

// One level: every entry of the frontier's lists, dealt out in block ranges of
// kLBS consecutive entries; the taken neighbours form the next frontier (one
// reservation per block range, so the counter is not a hot spot).
__global__ __launch_bounds__(256) void scc_expand(const uint32_t* front, const uint32_t* pre,
                                                  const int* row_off, const int* col,
                                                  const int* rrow_off, const int* rcol,
                                                  const uint32_t* live, const int* color,
                                                  int* flags, uint32_t* next,
                                                  unsigned long long* misc) {
    __shared__ uint32_t s_pre[kLBS + 1];
    __shared__ int s_start[kLBS + 1];
    __shared__ uint32_t s_item[kLBS + 1];
    __shared__ int s_cv[kLBS + 1];
    __shared__ uint32_t s_out[kLBS];
    __shared__ int s_nout;
    __shared__ unsigned long long s_base;
    const long long F = (long long)misc[kSccFront];
    const unsigned long long E = misc[kSccTotal];
    unsigned long long ors = 0;
    for (unsigned long long e0 = (unsigned long long)blockIdx.x * kLBS; e0 < E;
         e0 += (unsigned long long)gridDim.x * kLBS) {
        const unsigned long long e1 = e0 + kLBS < E ? e0 + kLBS : E;
        // the frontier items that own the range's first and last entries
        const long long o0 = owner_search(pre, F, e0);
        const long long o1 = owner_search(pre, F, e1 - 1);
        // Every frontier vertex is unassigned, so both of its lists are
        // non-empty: the owners of kLBS consecutive entries are at most kLBS.
        const int cnt = (int)min(o1 - o0 + 1, (long long)kLBS);
        if (threadIdx.x == 0) s_nout = 0;
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
            const uint32_t it = front[o0 + t];
            const int v = (int)(it & kIdMask);
            s_pre[t] = pre[o0 + t];
            s_item[t] = it;
            s_start[t] = ((it >> 30) ? rrow_off : row_off)[v];
            s_cv[t] = color ? color[v] : 0;
        }
        __syncthreads();
#pragma unroll 2
        for (int j = 0; j < kLBS / 256; ++j) {
            const unsigned long long e = e0 + (unsigned long long)j * 256 + threadIdx.x;
            if (e < e1) {
                int lo = 0, hi = cnt - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((unsigned long long)s_pre[mid] <= e) lo = mid;
                    else hi = mid - 1;
                }
                const uint32_t it = s_item[lo];
                const int dir = (int)(it >> 30);
                const int w = (dir ? rcol : col)[s_start[lo] + (int)(e - s_pre[lo])];
                bool tried;
                if (take(w, dir ? 2 : 1, s_cv[lo], live, color, flags, tried))
                    s_out[atomicAdd(&s_nout, 1)] = ritem(dir, w);
                ors += tried;
            }
        }
        __syncthreads();
        const int nout = s_nout;
        if (nout > 0) {
            if (threadIdx.x == 0)
                s_base = __hip_atomic_fetch_add(misc + kSccNext, (unsigned long long)nout,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const unsigned long long base = s_base;
            for (int t = threadIdx.x; t < nout; t += blockDim.x) next[base + t] = s_out[t];
        }
        __syncthreads();
    }
    ors = wave_sum(ors);
    if (lane_id() == 0 && ors) add_misc(misc + kSccOrs, ors);
}

// Size-2 check (the pattern after size-1 trimming): the only remaining
// neighbour of u in one list, or -1 when u has none, several, or itself.
__device__ __forceinline__ int only_neighbour(const int* off, const int* adj, int u,
                                              const uint32_t* live) {
    int a = -1;
    const int e = off[u + 1];
    for (int p = off[u]; p < e; ++p) {
        const int w = adj[p];
        if (!has_bit(live, w)) continue;
        if (w == u || (a >= 0 && w != a)) return -1;
        a = w;
    }
    return a;
}

__global__ void size2_only(int n, const int* row_off, const int* col, const int* rrow_off,
                           const int* rcol, const uint32_t* live, int* only_in, int* only_out) {
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        const bool a = has_bit(live, u);
        only_in[u] = a ? only_neighbour(rrow_off, rcol, u, live) : -1;
        only_out[u] = a ? only_neighbour(row_off, col, u, live) : -1;
    }
}

// partner[u] = v when u and v are each other's only remaining predecessor
// (nothing else reaches the pair) or only remaining successor (the pair
// reaches nothing else): a component of two.  -1 otherwise.
__global__ void size2_pair(int n, const int* only_in, const int* only_out, int* partner) {
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        int p = -1;
        const int a = only_in[u], b = only_out[u];
        if (a >= 0 && only_in[a] == u) p = a;
        else if (b >= 0 && only_out[b] == u) p = b;
        partner[u] = p;
    }
}

__global__ void size2_count(int n, const int* partner, unsigned long long* misc) {
    __shared__ unsigned long long red[16];
    unsigned long long c = 0;
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x)
        c += partner[u] >= 0;
    c = block_total(c, red);
    if (threadIdx.x == 0 && c) add_misc(misc + kSccCount, c);
}

// Paired vertices join their component, labelled with the pair's smaller id.
__global__ void scc_take_pairs(int n, const uint32_t* live, const int* partner, int* label,
                               uint32_t* assigned, unsigned long long* misc) {
    __shared__ unsigned long long red[16];
    const int waves = (gridDim.x * blockDim.x) / kWave;
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    unsigned long long taken = 0;
    for (int base = wid * kWave; base < n; base += waves * kWave) {
        const int v = base + lane_id();
        const int p = v < n && has_bit(live, v) ? partner[v] : -1;
        if (p >= 0) label[v] = min(v, p);
        const uint64_t m = ballot(p >= 0);
        if (lane_id() == 0 && m) {
            assigned[base >> 5] |= (uint32_t)m;
            assigned[(base >> 5) + 1] |= (uint32_t)(m >> 32);
            taken += (unsigned long long)popc(m);
        }
    }
    taken = block_total(taken, red);
    if (threadIdx.x == 0 && taken) add_misc(misc + kSccTaken, taken);
}

// live = not preset (all vertices when preset is NULL), bits past n clear.
__global__ void scc_live_from_preset(int n, const uint32_t* preset, uint32_t* live) {
    const int words = (n + 31) >> 5;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < words; w += gridDim.x * blockDim.x) {
        const uint32_t valid = (w == words - 1 && (n & 31)) ? ((1u << (n & 31)) - 1u) : ~0u;
        live[w] = (preset ? ~preset[w] : ~0u) & valid;
    }
}

// After a level: the next frontier becomes the current one.
__global__ void scc_level_done(unsigned long long* misc) {
    if (threadIdx.x == 0) {
        misc[kSccFront] = misc[kSccNext];
        misc[kSccLevels] += 1;
    }
}

// Unassigned vertices with the wanted marks join a component: mode 0 (both
// marks) gets the pivot's id, mode 1 (backward mark) the colour (its root).
// One wavefront per 64 consecutive vertices, so each assigned word has one
// writer.
__global__ void scc_take_marked(int n, int mode, const uint32_t* live, const int* flags,
                                const int* color, int* label, uint32_t* assigned,
                                unsigned long long* misc) {
    __shared__ unsigned long long red[16];
    const int pivot = (int)(misc[kSccPivot] & 0xFFFFFFFFull);
    const int waves = (gridDim.x * blockDim.x) / kWave;
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    unsigned long long taken = 0;
    for (int base = wid * kWave; base < n; base += waves * kWave) {
        const int v = base + lane_id();
        bool in = false;
        if (v < n && has_bit(live, v)) {
            const int f = flags[v];
            in = mode == 0 ? f == 3 : (f & 2) != 0;
            if (in) label[v] = mode == 0 ? pivot : color[v];
        }
        const uint64_t m = ballot(in);
        if (lane_id() == 0 && m) {
            assigned[base >> 5] |= (uint32_t)m;
            assigned[(base >> 5) + 1] |= (uint32_t)(m >> 32);
            taken += (unsigned long long)popc(m);
        }
    }
    taken = block_total(taken, red);
    if (threadIdx.x == 0 && taken) add_misc(misc + kSccTaken, taken);
}

__global__ void scc_count_reps(int n, const int* label, unsigned long long* misc) {
    __shared__ unsigned long long red[16];
    unsigned long long c = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        c += label[v] == v;
    c = block_total(c, red);
    if (threadIdx.x == 0 && c) add_misc(misc + kSccCount, c);
}

inline int grid_for(long long n, int block, int max_blocks = 1 << 20) {
    long long b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

}  // namespace

hipError_t scc_run(const trim_csr_t& g, const Work& w, const Work2& x, const SccWork& s,
                   const LaunchCfg& lc, int* label, SccCounts* counts) {
    const int n = g.n;
    hipStream_t st = lc.stream;
    const int gv = grid_for(n, 256, lc.cus * 8);
    const int gw = grid_for((n + 31) / 32, 256, lc.cus * 8);
    unsigned long long host[kSccMisc];
    hipError_t e;
    auto read_misc = [&]() -> hipError_t {
        hipError_t r = hipMemcpyAsync(host, s.misc, sizeof host, hipMemcpyDeviceToHost, st);
        if (r == hipSuccess) r = hipStreamSynchronize(st);
        return r;
    };
    auto reset = [&](int mask) {
        hipLaunchKernelGGL(scc_reset, dim3(1), dim3(256), 0, st, s.misc, mask, w.ctr);
    };
    // level-synchronous search from the items in front[0] (misc[kSccFront] of
    // them); ends when a level takes nothing
    auto search = [&](const int* color) -> hipError_t {
        const int ge = lc.cus * 8;
        for (int cur = 0;; cur ^= 1) {
            hipLaunchKernelGGL(scc_scan_chunks, dim3(ge), dim3(256), 0, st, s.front[cur],
                               g.row_off, g.rrow_off, s.pre, s.bsum, s.misc);
            hipLaunchKernelGGL(scc_scan_sums, dim3(1), dim3(1024), 0, st, s.bsum, s.misc);
            hipLaunchKernelGGL(scc_scan_add, dim3(ge), dim3(256), 0, st, s.pre, s.bsum, s.misc);
            hipLaunchKernelGGL(scc_expand, dim3(ge), dim3(256), 0, st, s.front[cur], s.pre,
                               g.row_off, g.col, g.rrow_off, g.rcol, s.live, color, s.flags,
                               s.front[cur ^ 1], s.misc);
            hipLaunchKernelGGL(scc_level_done, dim3(1), dim3(64), 0, st, s.misc);
            hipError_t r = hipGetLastError();
            if (r == hipSuccess) r = read_misc();
            if (r != hipSuccess) return r;
            if (host[kSccFront] == 0) break;
        }
        return hipSuccess;
    };
    using clock = std::chrono::steady_clock;
    auto ms_since = [](clock::time_point t0) {
        return std::chrono::duration<double, std::milli>(clock::now() - t0).count();
    };
    // two-sided trim of the unassigned vertices; returns how many remain
    long long active = 0;
    auto trim_round = [&]() -> hipError_t {
        const auto t0 = clock::now();
        hipError_t r = ac6_two_csr_preset(g, w, x, lc, s.live, w.wedges, nullptr, s.assigned);
        if (r != hipSuccess) return r;
        reset((1 << kSccActive) | (1 << kSccTaken));
        hipLaunchKernelGGL(scc_take_trimmed, dim3(gw), dim3(256), 0, st, n, s.live, s.assigned,
                           label, s.misc);
        if ((r = hipGetLastError()) != hipSuccess || (r = read_misc()) != hipSuccess) return r;
        active = (long long)host[kSccActive];
        int stalled = 0;   // the trimming pass was abandoned by its watchdog
        if ((r = hipMemcpyAsync(&stalled, w.ctr + kStall, sizeof(int), hipMemcpyDeviceToHost,
                                st)) != hipSuccess ||
            (r = hipStreamSynchronize(st)) != hipSuccess)
            return r;
        if (stalled) {
            counts->stalled = true;
            active = 0;
        }
        counts->trimmed += (long long)host[kSccTaken];
        counts->trims += 1;
        counts->trim_ms += ms_since(t0);
        return hipSuccess;
    };

    hipLaunchKernelGGL(scc_init, dim3(gv), dim3(256), 0, st, n, label, s.flags, s.assigned, s.misc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    if ((e = trim_round()) != hipSuccess) return e;
    if (active > 0) {
        // the pivot's component by forward-backward search
        const auto t0 = clock::now();
        reset((1 << kSccPivot) | (1 << kSccTaken));
        hipLaunchKernelGGL(scc_pivot, dim3(gv), dim3(256), 0, st, n, g.row_off, g.rrow_off, s.live,
                           s.misc);
        hipLaunchKernelGGL(scc_seed_pivot, dim3(1), dim3(64), 0, st, s.misc, s.flags,
                           s.front[0]);
        if ((e = search(nullptr)) != hipSuccess) return e;
        hipLaunchKernelGGL(scc_take_marked, dim3(gv), dim3(256), 0, st, n, 0, s.live, s.flags,
                           (const int*)nullptr, label, s.assigned, s.misc);
        if ((e = hipGetLastError()) != hipSuccess || (e = read_misc()) != hipSuccess) return e;
        counts->giant = (long long)host[kSccTaken];
        counts->search_ms += ms_since(t0);
        if ((e = trim_round()) != hipSuccess) return e;
    }
    if (active > 0) {
        // size-2 components (each the other's only remaining predecessor or
        // successor), then trimming again if any were found
        const auto t0 = clock::now();
        int* partner = reinterpret_cast<int*>(s.pre);
        reset(1 << kSccTaken);
        hipLaunchKernelGGL(size2_only, dim3(gv), dim3(256), 0, st, n, g.row_off, g.col, g.rrow_off,
                           g.rcol, s.live, s.flags, s.color);
        hipLaunchKernelGGL(size2_pair, dim3(gv), dim3(256), 0, st, n, s.flags, s.color, partner);
        hipLaunchKernelGGL(scc_take_pairs, dim3(gv), dim3(256), 0, st, n, s.live, partner, label,
                           s.assigned, s.misc);
        if ((e = hipGetLastError()) != hipSuccess || (e = read_misc()) != hipSuccess) return e;
        counts->paired = (long long)host[kSccTaken];
        counts->size2_ms += ms_since(t0);
        if (counts->paired > 0 && (e = trim_round()) != hipSuccess) return e;
    }
    while (active > 0) {
        // colouring round
        const auto t0 = clock::now();
        hipLaunchKernelGGL(scc_color_init, dim3(gv), dim3(256), 0, st, n, s.live, s.color, s.flags);
        for (long long sweep = 0;; ++sweep) {
            if (sweep > (long long)n + 1) {   // a colour travels at most n - 1 edges
                counts->stalled = true;
                return hipSuccess;
            }
            reset(1 << kSccChanged);
            hipLaunchKernelGGL(scc_color_sweep, dim3(gv), dim3(256), 0, st, n, g.row_off, g.col,
                               s.live, s.color, s.misc);
            if ((e = hipGetLastError()) != hipSuccess || (e = read_misc()) != hipSuccess) return e;
            counts->color_sweeps += 1;
            if (host[kSccChanged] == 0) break;
        }
        reset((1 << kSccTaken) | (1 << kSccFront));
        hipLaunchKernelGGL(scc_seed_roots, dim3(gv), dim3(256), 0, st, n, s.live, s.color, s.flags,
                           s.front[0], s.misc);
        if ((e = search(s.color)) != hipSuccess) return e;
        hipLaunchKernelGGL(scc_take_marked, dim3(gv), dim3(256), 0, st, n, 1, s.live, s.flags,
                           (const int*)s.color, label, s.assigned, s.misc);
        if ((e = hipGetLastError()) != hipSuccess || (e = read_misc()) != hipSuccess) return e;
        if (host[kSccTaken] == 0) {   // a round always takes at least its roots
            counts->stalled = true;
            return hipSuccess;
        }
        counts->color_rounds += 1;
        counts->color_ms += ms_since(t0);
        if ((e = trim_round()) != hipSuccess) return e;
    }
    reset(1 << kSccCount);
    hipLaunchKernelGGL(scc_count_reps, dim3(gv), dim3(256), 0, st, n, label, s.misc);
    if ((e = hipGetLastError()) != hipSuccess || (e = read_misc()) != hipSuccess) return e;
    counts->n_scc = (long long)host[kSccCount];
    counts->search_edges = (long long)host[kSccEdges];
    counts->search_levels = (int)host[kSccLevels];
    counts->search_ors = (long long)host[kSccOrs];
    return hipSuccess;
}



}  // namespace trim

namespace trim {

hipError_t size2_run(const trim_csr_t& g, const SccWork& s, const uint32_t* preset, int* partner,
                     long long* n_paired, hipStream_t st, int cus) {
    const int n = g.n;
    if (n_paired) *n_paired = 0;
    if (n == 0) return hipSuccess;
    const int gv = grid_for(n, 256, cus * 8);
    const int gw = grid_for((n + 31) / 32, 256, cus * 8);
    hipLaunchKernelGGL(scc_live_from_preset, dim3(gw), dim3(256), 0, st, n, preset, s.live);
    hipLaunchKernelGGL(size2_only, dim3(gv), dim3(256), 0, st, n, g.row_off, g.col, g.rrow_off,
                       g.rcol, s.live, s.flags, s.color);
    hipLaunchKernelGGL(size2_pair, dim3(gv), dim3(256), 0, st, n, s.flags, s.color, partner);
    if (n_paired) {
        unsigned long long c = 0;
        hipLaunchKernelGGL(scc_reset, dim3(1), dim3(256), 0, st, s.misc, 1 << kSccCount,
                           (int*)nullptr);
        hipLaunchKernelGGL(size2_count, dim3(gv), dim3(256), 0, st, n, partner, s.misc);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(&c, s.misc + kSccCount, sizeof c, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        *n_paired = (long long)c;
    }
    return hipGetLastError();
}

}  // namespace trim
