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
// label[v] is the id of one vertex of v's component (v itself, the pivot or
// the root); equal labels mean one component.
//
// The searches run in one persistent launch each, on the same per-wavefront
// LDS rings and shared queue as the trimming kernels (WaveQueue): an item is
// a vertex to expand forward (successors) or backward (predecessors); a
// neighbour is taken once per direction, by the lane whose fetch-or sets its
// mark first.
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

// Zeroes the misc words selected by `mask` and the queue counters (one block).
__global__ void scc_reset(unsigned long long* misc, int mask, int* ctr) {
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

// The pivot, marked and queued in both directions (one block, counters zeroed
// by scc_reset before).
__global__ void scc_seed_pivot(const unsigned long long* misc, int* flags, uint32_t* q, int* ctr) {
    if (threadIdx.x == 0) {
        const int v = (int)(misc[kSccPivot] & 0xFFFFFFFFull);
        flags[v] = 3;
        q[0] = ritem(0, v);
        q[1] = ritem(1, v);
        ctr[kQTail] = 2;
        ctr[kPending] = 2;
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

// Roots (unassigned v with colour v): marked backward and queued backward
// (counters zeroed by scc_reset before).
__global__ void scc_seed_roots(int n, const uint32_t* live, const int* color, int* flags,
                               uint32_t* q, int* ctr) {
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int v = base + threadIdx.x;
        const bool root = v < n && has_bit(live, v) && color[v] == v;
        if (root) flags[v] = 2;
        const int slot = wave_append_slot(root, ctr + kQTail, ctr + kPending);
        if (root) q[slot] = ritem(1, v);
    }
}

constexpr int kRBatch = 8;
constexpr int kRCoop = 32;   // lists longer than this are expanded by the whole wavefront

// Takes w for direction bit `bit` if it is unassigned, in colour c (when
// colours are used) and not yet marked: the fetch-or that sets the mark wins.
__device__ __forceinline__ bool take(int w, int bit, int c, const uint32_t* live, const int* color,
                                     int* flags) {
    if (!has_bit(live, w)) return false;
    if (color && color[w] != c) return false;
    if (ld_cached(flags + w) & bit) return false;
    return (or_dev(flags + w, bit) & bit) == 0;
}

// Forward / backward search from the queued items, inside the unassigned
// vertices (and inside one colour when `color` is given).
__global__ __launch_bounds__(256) void scc_reach(const int* row_off, const int* col,
                                                 const int* rrow_off, const int* rcol,
                                                 const uint32_t* live, const int* color,
                                                 int* flags, uint32_t* q, int* ctr,
                                                 unsigned long long* misc) {
    __shared__ uint32_t rings[256 / kWave][kLocalQ];
    __shared__ int ring_tail[256 / kWave];
    WaveQueue wq;
    const int wv = threadIdx.x / kWave;
    wq.init(rings[wv], &ring_tail[wv], q, ctr + kQHead, ctr + kQTail, ctr + kPending);
    uint32_t item = kNone;
    int k = 0, e = 0, dir = 0, cv = 0;
    bool started = false;
    uint64_t examined = 0;
    while (wq.acquire(item)) {
        uint32_t out[kRBatch];
#pragma unroll
        for (int j = 0; j < kRBatch; ++j) out[j] = kNone;
        if (item != kNone && !started) {
            const int v = (int)(item & kIdMask);
            dir = (int)(item >> 30);
            const int* off = dir ? rrow_off : row_off;
            k = off[v];
            e = off[v + 1];
            cv = color ? color[v] : 0;
            started = true;
            examined += (uint64_t)(e - k);
        }
        for (uint64_t big = ballot(item != kNone && e - k > kRCoop); big; big &= big - 1) {
            const int owner = __ffsll((unsigned long long)big) - 1;
            const int kb = __shfl(k, owner), eb = __shfl(e, owner);
            const int db = __shfl(dir, owner), cb = __shfl(cv, owner);
            const int* adj = db ? rcol : col;
            const int bit = db ? 2 : 1;
            for (int base = kb; base < eb; base += kWave * kRBatch) {
                int u[kRBatch];
                uint32_t o[kRBatch];
#pragma unroll
                for (int j = 0; j < kRBatch; ++j) {
                    const int p = base + j * kWave + lane_id();
                    if (p < eb) u[j] = adj[p];
                }
#pragma unroll
                for (int j = 0; j < kRBatch; ++j) {
                    const int p = base + j * kWave + lane_id();
                    o[j] = (p < eb && take(u[j], bit, cb, live, color, flags)) ? ritem(db, u[j])
                                                                              : kNone;
                }
#pragma unroll
                for (int j = 0; j < kRBatch; j += 2) wq.push(o[j], o[j + 1]);
            }
            if (lane_id() == owner) {
                item = kNone;
                started = false;
            }
        }
        if (item != kNone) {
            const int nb = min(kRBatch, e - k);
            const int* adj = dir ? rcol : col;
            const int bit = dir ? 2 : 1;
            int u[kRBatch];
#pragma unroll
            for (int j = 0; j < kRBatch; ++j)
                if (j < nb) u[j] = adj[k + j];
#pragma unroll
            for (int j = 0; j < kRBatch; ++j)
                if (j < nb && take(u[j], bit, cv, live, color, flags)) out[j] = ritem(dir, u[j]);
            k += nb;
            if (k >= e) {
                item = kNone;
                started = false;
                // depth first: go on with a vertex this lane has just taken
#pragma unroll
                for (int j = 0; j < kRBatch; ++j)
                    if (item == kNone && out[j] != kNone) {
                        item = out[j];
                        out[j] = kNone;
                    }
            }
        }
#pragma unroll
        for (int j = 0; j < kRBatch; j += 2) wq.push(out[j], out[j + 1]);
        wq.rebalance();
    }
    examined = wave_sum(examined);
    if (lane_id() == 0 && examined) add_misc(misc + kSccEdges, examined);
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
        hipLaunchKernelGGL(scc_seed_pivot, dim3(1), dim3(64), 0, st, s.misc, s.flags, w.q, w.ctr);
        hipLaunchKernelGGL(scc_reach, dim3(lc.workers), dim3(256), 0, st, g.row_off, g.col,
                           g.rrow_off, g.rcol, s.live, (const int*)nullptr, s.flags, w.q, w.ctr,
                           s.misc);
        hipLaunchKernelGGL(scc_take_marked, dim3(gv), dim3(256), 0, st, n, 0, s.live, s.flags,
                           (const int*)nullptr, label, s.assigned, s.misc);
        if ((e = hipGetLastError()) != hipSuccess || (e = read_misc()) != hipSuccess) return e;
        counts->giant = (long long)host[kSccTaken];
        counts->search_ms += ms_since(t0);
        if ((e = trim_round()) != hipSuccess) return e;
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
        reset(1 << kSccTaken);
        hipLaunchKernelGGL(scc_seed_roots, dim3(gv), dim3(256), 0, st, n, s.live, s.color, s.flags,
                           w.q, w.ctr);
        hipLaunchKernelGGL(scc_reach, dim3(lc.workers), dim3(256), 0, st, g.row_off, g.col,
                           g.rrow_off, g.rcol, s.live, (const int*)s.color, s.flags, w.q, w.ctr,
                           s.misc);
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
    return hipSuccess;
}

int scc_max_workers_per_cu(int) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, scc_reach, 256, 0) != hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

}  // namespace trim
