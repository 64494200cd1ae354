// batch.hip -- trim_batch: AC-6 over a batch of independent graphs, each graph
// owned by one workgroup (Section 6.2, Alg. par-ac-6-trim, run per graph).
//
// The graphs of a batch share nothing, so a graph needs no device-wide
// coordination at all: one workgroup claims it, trims it start to finish and
// claims the next.  Claims go largest first (graphs ordered by the size class
// of n + m), so the biggest graphs start early and the small ones fill in
// behind them.  Within a graph the AC-6 steps are those of the one-graph path:
//   init   both list heads kDead (no successor) or kEmpty;
//   sweep  DoPost for every vertex: the first successor that is not a sink
//          becomes its support (join: exchange into the support's S_more or
//          S_last head, whichever its position selects); vertices with none
//          become CLOSE items;
//   phases each phase takes the list the previous one built: CLOSE(x)
//          exchanges both heads of x with kDead and walks the two lists it
//          got back -- every S_last member is removed with x (a CLOSE item
//          for the next phase), every S_more member resumes its scan after
//          its old support (a RESCAN item); RESCAN(x) resumes x's scan and
//          closes x on the spot if it finds nothing.  A workgroup barrier
//          ends a phase; the graph is done when a phase builds an empty list.
//   pack   the graph's own bitmap words, its live count, its traversed-edge
//          total (exact: one workgroup makes all of the graph's checks).
// Items and list counters live in LDS; heads, records and the two phase lists
// of a graph live in device memory at the graph's own vertex range, where the
// workgroup's L2 keeps them for the graph's lifetime.
#include "trim_internal.h"
#include "trim_device.h"
#include "trim_stats.h"
#include "ac6_support.h"

namespace trim {
namespace {

// One graph of the batch: global vertex ids vb + local id.
struct OwnedView {
    const int* row_off;
    const int* col;
    int vb;
    __device__ __forceinline__ int vctx(int) const { return vb; }
    __device__ __forceinline__ int begin(int v) const { return row_off[v]; }
    __device__ __forceinline__ int end(int v) const { return row_off[v + 1]; }
    __device__ __forceinline__ int target(int, int p, int b) const { return b + col[p]; }
};

enum : uint32_t { kOwnClose = 0, kOwnRescan = 1 };
constexpr int kOwnMaxBlock = 1024;
constexpr int kOwnStage = 128;    // items staged per wavefront before one reservation
constexpr int kOwnUnroll = 2;     // sweep vertices per lane in flight
// Graphs with n + m >= 2^15 are trimmed by a whole workgroup, smaller ones by
// one wavefront each (size_key is the count of leading zeros of n + m).
constexpr int kBigKey = 31 - 15;

// Size class of graph gi: larger graphs get smaller keys.
__device__ __forceinline__ int size_key(const int64_t* vbase, const int* row_off, int gi) {
    const int64_t v0 = vbase[gi], v1 = vbase[gi + 1];
    const uint32_t size = (uint32_t)(row_off[v1] - row_off[v0]) + (uint32_t)(v1 - v0);
    return __clz(size > 0 ? size : 1u);
}

// One block: order[] = graph indices by descending size class; zeroes the
// control words and the statistics.
__global__ void batch_order(const int64_t* vbase, const int* row_off, int G, int* order, int* ctr,
                            trim_stats_t* stats) {
    __shared__ int hist[33];
    for (int i = threadIdx.x; i < kCtrInts; i += blockDim.x) ctr[i] = 0;
    if (stats && threadIdx.x < (int)(sizeof(trim_stats_t) / 8))
        ((uint64_t*)stats)[threadIdx.x] = 0;
    if (threadIdx.x < 33) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int gi = threadIdx.x; gi < G; gi += blockDim.x)
        atomicAdd(&hist[size_key(vbase, row_off, gi)], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < 33; ++k) {
            const int c = hist[k];
            hist[k] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int gi = threadIdx.x; gi < G; gi += blockDim.x)
        order[atomicAdd(&hist[size_key(vbase, row_off, gi)], 1)] = gi;
}

// Every word of a graph's state (heads, records, phase lists) is touched by
// its owning workgroup only, so workgroup-scope accesses keep it coherent;
// the workgroup's L2 serves them.
constexpr int kWG = __HIP_MEMORY_SCOPE_WORKGROUP;

// Dead-vertex bitmap of an owned graph in LDS: a bit per local vertex, set for
// sinks at init and by every close.  Successor checks read it instead of a
// list head in device memory (a random cache line per check); a join still
// reads the head and its CAS fails on kDead, so a bit that is not yet set
// only costs that attempt.  kBitsWords words per workgroup: the whole array
// for a workgroup's graph, an equal share per wavefront for wavefront graphs.
constexpr int kBitsWords = 16384;   // 64 KiB: 2^19 vertices

// Shared state of an owned-graph kernel's workgroup (LDS).
struct OwnShared {
    uint32_t bits[kBitsWords];
    uint32_t stage[kOwnMaxBlock / kWave][kOwnStage];   // per-wavefront item staging
    int stage_n[kOwnMaxBlock / kWave];
    int cnt[kOwnMaxBlock / kWave];   // items in the list being built: [0] for the
                                     // workgroup, [wave] for a wavefront's own graph
    int claim;
    uint64_t red[16];
};

// Per-thread running totals of the kernel.
struct OwnTotals {
    uint64_t edges = 0, sweep = 0, closes = 0, joins = 0, visited = 0, live = 0, deg = 0;
    int max_phases = 0;
};

__device__ __forceinline__ bool bit_dead(const uint32_t* bits, int l) {
    return (bits[l >> 5] >> (l & 31)) & 1u;
}

// Resume DoPost of u (global id) from position p0, skipping targets whose
// bit is set; as resume() otherwise (the same checks are counted).
__device__ __forceinline__ bool resume_own(const OwnedView& g, int u, int p0, int* head,
                                           uint64_t* rec, uint64_t& edges, int sched,
                                           const uint32_t* bits) {
    constexpr int kScan = 8;
    const int e = g.end(u);
    for (int p = p0; p < e; p += kScan) {
        int w[kScan];
#pragma unroll
        for (int j = 0; j < kScan; ++j)
            if (p + j < e) w[j] = g.col[p + j];
#pragma unroll
        for (int j = 0; j < kScan; ++j) {
            if (p + j >= e) break;
            if (bit_dead(bits, w[j])) continue;
            int* slot = head + 2 * (g.vb + w[j]) + (p + j + 1 == e);
            int hj = ld_s<kWG>(slot);
            while (hj != kDead) {
                st_s<kWG>(rec + u, pack_rec(hj, p + j));
                complete_mem();
                if (sched & TRIM_SCHED_JITTER) jitter_nap(((uint64_t)u << 24) ^ (p + j));
                if (cas_s<kWG>(slot, hj, u)) {
                    edges += (uint64_t)(p + j - p0 + 1);
                    return true;
                }
            }
        }
    }
    edges += (uint64_t)(e - p0);
    return false;
}

// Trim graph gi with a group of threads: the whole workgroup (kWaveGroup
// false; phases end at workgroup barriers) or one wavefront (true; its lanes
// run in lock step, so a phase ends with the wavefront's own memory wait).
// `bits`: the group's LDS bitmap, or nullptr if the graph does not fit it
// (then statuses are read from the heads).
template <bool kWaveGroup>
__device__ void own_graph(int gi, const int64_t* vbase, const int* row_off, const int* col,
                          const int64_t* bitmap_base, int* head, uint64_t* rec, uint32_t* l0,
                          uint32_t* l1, uint32_t* bitmaps, uint64_t* graph_edges, int sched,
                          OwnShared& sh, OwnTotals& t, uint32_t* bits) {
    const int wv = threadIdx.x / kWave;
    const int rank = kWaveGroup ? lane_id() : (int)threadIdx.x;
    const int size = kWaveGroup ? kWave : (int)blockDim.x;
    int* cnt = kWaveGroup ? &sh.cnt[wv] : &sh.cnt[0];
    auto sync = [&]() {
        complete_mem();
        if (kWaveGroup)
            __builtin_amdgcn_wave_barrier();
        else
            __syncthreads();
    };
    const int vb = (int)vbase[gi], ve = (int)vbase[gi + 1];
    const OwnedView g{row_off, col, vb};
    uint32_t* out = nullptr;
    // move this wavefront's staged items to the list being built (wave-uniform)
    auto flush = [&]() {
        const int k = sh.stage_n[wv];
        if (k == 0) return;
        int base = 0;
        if (lane_id() == 0) base = atomicAdd(cnt, k);
        base = __shfl(base, 0);
        for (int i = lane_id(); i < k; i += kWave) out[base + i] = sh.stage[wv][i];
        __builtin_amdgcn_wave_barrier();
        if (lane_id() == 0) sh.stage_n[wv] = 0;
        __builtin_amdgcn_wave_barrier();
    };
    // stage this lane's item, if any (wave-uniform)
    auto emit = [&](uint32_t it) {
        const uint64_t mk = ballot(it != kNone);
        const int k = popc(mk);
        if (k == 0) return;
        if (sh.stage_n[wv] + k > kOwnStage) flush();
        const int base = sh.stage_n[wv];
        if (it != kNone) sh.stage[wv][base + popc(mk & lanes_below())] = it;
        __builtin_amdgcn_wave_barrier();
        if (lane_id() == 0) sh.stage_n[wv] = base + k;
        __builtin_amdgcn_wave_barrier();
    };
    uint64_t edges = 0;
    // init: the heads of the graph's vertices and the sinks' bits (one word of
    // the bitmap per 32 local vertices: a lane ORs its vertex's bit in)
    if (bits)
        for (int i = rank; i < ((ve - vb + 31) >> 5); i += size) bits[i] = 0;
    sync();
    for (int v = vb + rank; v < ve; v += size) {
        const int b = row_off[v], e = row_off[v + 1];
        const int h = b == e ? kDead : kEmpty;
        reinterpret_cast<int2*>(head)[v] = make_int2(h, h);
        if (bits && b == e) atomicOr(&bits[(v - vb) >> 5], 1u << ((v - vb) & 31));
        t.deg += (uint64_t)(e - b);
    }
    if (rank == 0) *cnt = 0;
    sync();
    // sweep: only sinks are removed while it runs, so a target is live iff it
    // has a successor
    auto sink = [&](int w) {
        return bits ? bit_dead(bits, w - vb) : row_off[w] == row_off[w + 1];
    };
    out = l0 + vb;
    for (int base = vb; base < ve; base += kOwnUnroll * size) {
        int v[kOwnUnroll], b[kOwnUnroll], e[kOwnUnroll], p[kOwnUnroll], w[kOwnUnroll];
        bool ok[kOwnUnroll];
#pragma unroll
        for (int k = 0; k < kOwnUnroll; ++k) {
            v[k] = base + k * size + rank;
            b[k] = e[k] = 0;
            if (v[k] < ve) {
                b[k] = row_off[v[k]];
                e[k] = row_off[v[k] + 1];
            }
            p[k] = b[k];
            w[k] = b[k] < e[k] ? vb + col[b[k]] : vb;
        }
#pragma unroll
        for (int k = 0; k < kOwnUnroll; ++k) {
            ok[k] = b[k] < e[k] && !sink(w[k]);
            if (b[k] < e[k] && !ok[k]) {
                for (++p[k]; p[k] < e[k]; ++p[k]) {
                    w[k] = vb + col[p[k]];
                    if (!sink(w[k])) break;
                }
                ok[k] = p[k] < e[k];
            }
        }
        int old[kOwnUnroll];
#pragma unroll
        for (int k = 0; k < kOwnUnroll; ++k) {
            if (ok[k]) {
                if (sched & TRIM_SCHED_JITTER) jitter_nap(((uint64_t)gi << 32) ^ (uint32_t)v[k]);
                old[k] = xchg_s<kWG>(head + 2 * w[k] + (p[k] + 1 == e[k]), v[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < kOwnUnroll; ++k) {
            uint32_t it = kNone;
            if (ok[k]) {
                st_s<kWG>(rec + v[k], pack_rec(old[k], p[k]));
                edges += (uint64_t)(p[k] - b[k] + 1);
            } else if (b[k] < e[k]) {
                it = make_item(kOwnClose, v[k]);
                edges += (uint64_t)(e[k] - b[k]);
            }
            emit(it);
        }
    }
    flush();
    t.sweep += edges;
    sync();
    // phases
    uint32_t* in = l0 + vb;
    out = l1 + vb;
    int ph = 0;
    for (int n_in = *cnt; n_in > 0; n_in = *cnt) {
        sync();   // every thread has read the count
        if (rank == 0) *cnt = 0;
        sync();
        ++ph;
        for (int base = 0; base < n_in; base += size) {
            const int i = base + rank;
            const uint32_t it = i < n_in ? (uint32_t)ld_s<kWG>((const int*)in + i) : kNone;
            int walk_last = -1, walk_more = -1, cx = -1;
            if (it != kNone) {
                const int x = item_vertex(it);
                if (item_kind(it) == kOwnRescan) {
                    // x is in no list until it joins again: its record is stable
                    const uint64_t r = ld_s<kWG>(rec + x);
                    if (sched & TRIM_SCHED_JITTER) jitter_nap((uint64_t)x);
                    const bool joined =
                        bits ? resume_own(g, x, rec_cursor(r) + 1, head, rec, edges, sched, bits)
                             : resume<OwnedView, kWG>(g, x, rec_cursor(r) + 1, head, rec, edges,
                                                      sched);
                    if (joined)
                        t.joins += 1;
                    else
                        cx = x;
                } else {
                    cx = x;
                }
            }
            if (cx >= 0) {
                if (sched & TRIM_SCHED_JITTER) jitter_nap((uint64_t)cx << 8);
                const int2 ab = xchg2_s<kWG>(head + 2 * cx, kDead, kDead);
                if (bits) atomicOr(&bits[(cx - vb) >> 5], 1u << ((cx - vb) & 31));
                t.closes += 1;
                walk_more = ab.x;
                walk_last = ab.y;
            }
            // a member's link is read before its item exists: its own
            // processing, in the next phase, is the only thing that can change
            // its record
            while (ballot(walk_last >= 0 || walk_more >= 0)) {
                uint32_t e = kNone;
                if (walk_last >= 0) {
                    const int nx = ld_s<kWG>(rec_link(rec, walk_last));
                    e = make_item(kOwnClose, walk_last);
                    walk_last = nx;
                } else if (walk_more >= 0) {
                    const int nx = ld_s<kWG>(rec_link(rec, walk_more));
                    e = make_item(kOwnRescan, walk_more);
                    walk_more = nx;
                }
                t.visited += e != kNone;
                emit(e);
            }
        }
        flush();
        sync();
        uint32_t* tmp = in;
        in = out;
        out = tmp;
    }
    t.max_phases = ph > t.max_phases ? ph : t.max_phases;
    // pack: the graph's bitmap words (bits past its n stay zero)
    const int64_t wb = bitmap_base[gi], we = bitmap_base[gi + 1];
    const int nwords = (ve - vb + 31) >> 5;
    if (bits) {
        for (int i = rank; i < nwords; i += size) {
            const int nb = ve - vb - 32 * i;   // vertices in this word
            const uint32_t valid = nb >= 32 ? 0xFFFFFFFFu : ((1u << nb) - 1u);
            const uint32_t word = ~bits[i] & valid;
            bitmaps[wb + i] = word;
            t.live += (uint64_t)__popc(word);
        }
    } else {
        const int gwave = kWaveGroup ? 0 : wv, gwaves = size / kWave;
        for (int base = vb + gwave * kWave; base < ve; base += gwaves * kWave) {
            const int v = base + lane_id();
            const uint64_t m = ballot(v < ve && ld_s<kWG>(head + 2 * v) != kDead);
            if (lane_id() == 0) {
                const int wi = (base - vb) >> 5;
                bitmaps[wb + wi] = (uint32_t)m;
                if (wi + 1 < nwords) bitmaps[wb + wi + 1] = (uint32_t)(m >> 32);
                t.live += (uint64_t)popc(m);
            }
        }
    }
    for (int64_t wi = wb + nwords + rank; wi < we; wi += size) bitmaps[wi] = 0;
    edges = kWaveGroup ? wave_sum(edges) : block_sum(edges, sh.red);
    if (rank == 0) {
        graph_edges[gi] = edges;
        t.edges += edges;
    }
    sync();
}

// Graphs are claimed in order (largest first).  A workgroup trims the graphs
// of at least kBigKey's size class together; once it claims a smaller one,
// its wavefronts go their own ways: each trims that graph or graphs it claims
// itself, so up to one small graph per wavefront is in flight.
__global__ __launch_bounds__(kOwnMaxBlock) void ac6_owned(
    const int64_t* vbase, const int* row_off, const int* col, const int64_t* bitmap_base, int G,
    const int* order, int* head, uint64_t* rec, uint32_t* l0, uint32_t* l1, int* ctr,
    uint32_t* bitmaps, uint64_t* graph_edges, uint64_t* wedges, uint64_t* part, int big_key,
    int sched) {
    __shared__ OwnShared sh;
    const int wv = threadIdx.x / kWave;
    if (lane_id() == 0) sh.stage_n[wv] = 0;
    OwnTotals t;
    int first = -1;   // the small graph that ended the workgroup's part, if any
    for (;;) {
        if (threadIdx.x == 0) sh.claim = add_dev(ctr + kCursor, 1);
        __syncthreads();
        const int claim = sh.claim;
        __syncthreads();
        if (claim >= G) break;
        const int gi = order[claim];
        if (size_key(vbase, row_off, gi) > big_key) {
            first = gi;
            break;
        }
        const int ng = (int)(vbase[gi + 1] - vbase[gi]);
        own_graph<false>(gi, vbase, row_off, col, bitmap_base, head, rec, l0, l1, bitmaps,
                         graph_edges, sched, sh, t,
                         ((ng + 31) >> 5) <= kBitsWords ? sh.bits : nullptr);
    }
    // wavefront part: wavefront 0 takes the graph that ended the workgroup part
    const int wave_words = kBitsWords / (blockDim.x / kWave);
    __syncthreads();   // the workgroup's bitmap is free for the wavefronts
    for (int gi = (wv == 0) ? first : -1;;) {
        if (gi < 0) {
            int c = 0;
            if (lane_id() == 0) c = add_dev(ctr + kCursor, 1);
            c = __shfl(c, 0);
            if (c >= G) break;
            gi = order[c];
        }
        const int ng = (int)(vbase[gi + 1] - vbase[gi]);
        own_graph<true>(gi, vbase, row_off, col, bitmap_base, head, rec, l0, l1, bitmaps,
                        graph_edges, sched, sh, t,
                        ((ng + 31) >> 5) <= wave_words ? sh.bits + wv * wave_words : nullptr);
        gi = -1;
    }
    __syncthreads();
    const uint64_t sweep = block_sum(t.sweep, sh.red);
    const uint64_t closes = block_sum(t.closes, sh.red);
    const uint64_t joins = block_sum(t.joins, sh.red);
    const uint64_t visited = block_sum(t.visited, sh.red);
    const uint64_t live = block_sum(t.live, sh.red);
    const uint64_t deg = block_sum(t.deg, sh.red);
    const uint64_t edges = block_sum(t.edges, sh.red);
    if (threadIdx.x == 0) {
        wedges[blockIdx.x] = edges;
        part[kPartSweep * kPartStride + blockIdx.x] = sweep;
        part[kPartDeg * kPartStride + blockIdx.x] = deg;
        part[kPartLive * kPartStride + blockIdx.x] = live;
        part[kPartLvCloses * kPartStride + blockIdx.x] = closes;
        part[kPartLvJoins * kPartStride + blockIdx.x] = joins;
        part[kPartLvVisited * kPartStride + blockIdx.x] = visited;
    }
    int mp = t.max_phases;
    for (int off = 32; off > 0; off >>= 1) mp = max(mp, __shfl_xor(mp, off));
    if (lane_id() == 0 && mp) atomicMax(ctr + kLvPhases, mp);
}

}  // namespace

int ac6_owned_blocks_per_cu(int block) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ac6_owned, block, 0) != hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

hipError_t ac6_batch_owned(int G, const int64_t* vbase, const int32_t* row_off,
                           const int32_t* col, int64_t total_n, const int64_t* bitmap_base,
                           const Work& w, const LaunchCfg& lc, uint32_t* bitmaps,
                           uint64_t* graph_edges, trim_stats_t* stats) {
    const int B = lc.block;
    int W = lc.workers > 0 ? lc.workers : lc.cus * ac6_owned_blocks_per_cu(B);
    if (W > kPartStride) W = kPartStride;
    {
        Timed t(lc, "batch_order");
        hipLaunchKernelGGL(batch_order, dim3(1), dim3(1024), 0, lc.stream, vbase, row_off, G, w.d,
                           w.ctr, stats);
    }
    {
        Timed t(lc, "ac6_owned");
        hipLaunchKernelGGL(ac6_owned, dim3(W), dim3(B), 0, lc.stream, vbase, row_off, col,
                           bitmap_base, G, w.d, w.a, w.b, w.e, w.e + w.cap, w.ctr, bitmaps,
                           graph_edges, w.wedges, w.part, kBigKey, lc.schedule);
    }
    if (stats) {
        Timed t(lc, "finalize");
        hipLaunchKernelGGL(finalize_stats, dim3(1), dim3(1024), 0, lc.stream, (int)total_n, W, W,
                           0, W, 0, w.wedges, w.part, w.ctr, stats, 0, 0, W);
    }
    return hipGetLastError();
}

}  // namespace trim
