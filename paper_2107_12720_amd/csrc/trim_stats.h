// Output and statistics kernels shared by the three propagation schemes: the
// live bitmap and the reduction of per-block partial sums into trim_stats_t.
#pragma once
#include "trim_device.h"

namespace trim {

// ---------------------------------------------------- outputs and statistics
// Per-block partial sums live in `part` (kPartStride words per quantity); one
// finalize block reduces them, so no word is updated by every block.

namespace {   // kernels below get a private copy in every translation unit

// Live bitmap (bit v%32 of word v/32) from a per-vertex predicate, by ballot.
// Also restores the shared queue (q, qwords; NULL for AC-3) if the watchdog
// abandoned the persistent kernel before it.
template <class IsLive>
__global__ void pack_bitmap(IsLive is_live, int n, uint32_t* bitmap, uint64_t* part,
                            const int* ctr, uint32_t* q, long long qwords) {
    __shared__ uint64_t red[16];
    clear_queue_if_stalled(ctr, q, qwords);
    const int nwords = (n + 31) >> 5;
    const int waves = (gridDim.x * blockDim.x) / kWave;
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    uint64_t live_cnt = 0;
    for (int base = wid * kWave; base < n; base += waves * kWave) {
        const int v = base + lane_id();
        const uint64_t b = ballot(v < n && is_live(v));
        if (lane_id() == 0) {
            const int w = base >> 5;
            bitmap[w] = (uint32_t)b;
            if (w + 1 < nwords) bitmap[w + 1] = (uint32_t)(b >> 32);
            live_cnt += (uint64_t)popc(b);
        }
    }
    live_cnt = block_sum(live_cnt, red);
    if (threadIdx.x == 0) part[kPartLive * kPartStride + blockIdx.x] = live_cnt;
}

__device__ __forceinline__ uint64_t sum_range(const uint64_t* a, int k, uint64_t* red) {
    uint64_t s = 0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) s += a[i];
    return block_sum(s, red);
}

__device__ __forceinline__ uint64_t max_range(const uint64_t* a, int k, uint64_t* red) {
    int m = 0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) m = max(m, (int)a[i]);
    return (uint64_t)block_max(m, reinterpret_cast<int*>(red));
}

// One block: reduce the partials into *stats.  n_sweep / n_prop = number of
// sweep / propagation partials (0 when the algorithm has none); n_qhw =
// number of ring high-water partials; n_live_edges = number of live-check
// partials (two-sided AC-6 only, else 0); n_levels = number of partials of
// the level-synchronous propagation phases (AC-6, else 0).
__global__ void finalize_stats(int n, int P, int n_sweep, int n_prop, int n_pack, int n_qhw,
                               const uint64_t* worker_edges, const uint64_t* part, const int* ctr,
                               trim_stats_t* stats, int empty_rounds, int n_live_edges = 0,
                               int n_levels = 0) {
    __shared__ uint64_t red[16];
    const uint64_t qhw = max_range(part + kPartQhw * kPartStride, n_qhw, red);
    const uint64_t edges = sum_range(worker_edges, P, red);
    const uint64_t live = sum_range(part + kPartLive * kPartStride, n_pack, red);
    const uint64_t sweep = sum_range(part + kPartSweep * kPartStride, n_sweep, red);
    // the propagation's counts: its level-synchronous phases and its asynchronous tail
    const uint64_t closes = sum_range(part + kPartCloses * kPartStride, n_prop, red) +
                            sum_range(part + kPartLvCloses * kPartStride, n_levels, red);
    const uint64_t joins = sum_range(part + kPartJoins * kPartStride, n_prop, red) +
                           sum_range(part + kPartLvJoins * kPartStride, n_levels, red);
    const uint64_t visited = sum_range(part + kPartVisited * kPartStride, n_prop, red) +
                             sum_range(part + kPartLvVisited * kPartStride, n_levels, red);
    const uint64_t degsum = sum_range(part + kPartDeg * kPartStride, n_sweep, red);
    const uint64_t live_edges = sum_range(part + kPartLiveEdges * kPartStride, n_live_edges, red);
    if (threadIdx.x == 0) {
        stats->edges_total = edges;
        stats->n_live = live;
        stats->n_dead = (uint64_t)n - live;
        stats->queued = (uint64_t)ctr[kQTail];
        stats->edges_sweep = sweep;
        stats->closes = closes;
        stats->joins = joins;
        stats->visited = visited;
        stats->graph_edges = degsum;
        stats->q_highwater = qhw;
        stats->edges_live = live_edges;
        stats->stalled = ld_dev(ctr + kStall) != 0;
        stats->forest = (uint64_t)ld_dev(ctr + kJKilled);
        stats->jump_rounds = (uint64_t)ld_dev(ctr + kJRounds);
        stats->work_items = (uint64_t)(uint32_t)ld_dev(ctr + kJWork) +
                            (uint64_t)(uint32_t)ld_dev(ctr + kAcWork);
        stats->phases = (uint64_t)ld_dev(ctr + kLvPhases);
        if (n == 0 && empty_rounds) stats->rounds = (uint64_t)empty_rounds;
    }
}

}  // namespace

}  // namespace trim
