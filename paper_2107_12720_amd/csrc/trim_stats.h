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

// One block: reduce the partials into *stats.  n_sweep / n_prop = number of
// sweep / propagation partials (0 when the algorithm has none); n_qhw =
// number of ring high-water partials; n_live_edges = number of live-check
// partials (two-sided AC-6 only, else 0); n_levels = number of partials of
// the level-synchronous propagation phases (AC-6, else 0).  Every thread
// sums its share of all quantities in one pass, and one reduction combines
// them (a reduction per quantity would cost a barrier pair each).
__global__ void finalize_stats(int n, int P, int n_sweep, int n_prop, int n_pack, int n_qhw,
                               const uint64_t* worker_edges, const uint64_t* part, const int* ctr,
                               trim_stats_t* stats, int empty_rounds, int n_live_edges = 0,
                               int n_levels = 0) {
    enum { kEdges, kLive, kSweep, kCloses, kJoins, kVisited, kDeg, kLiveE, kQhw, kN };
    __shared__ uint64_t red[kN][16];
    uint64_t acc[kN] = {};
    const auto P_ = [&](int slot, int i) { return part[slot * kPartStride + i]; };
    int most = P;
    for (int k : {n_sweep, n_prop, n_pack, n_qhw, n_live_edges, n_levels}) most = k > most ? k : most;
    for (int i = threadIdx.x; i < most; i += blockDim.x) {
        if (i < P) acc[kEdges] += worker_edges[i];
        if (i < n_pack) acc[kLive] += P_(kPartLive, i);
        if (i < n_sweep) {
            acc[kSweep] += P_(kPartSweep, i);
            acc[kDeg] += P_(kPartDeg, i);
        }
        if (i < n_prop) {
            acc[kCloses] += P_(kPartCloses, i);
            acc[kJoins] += P_(kPartJoins, i);
            acc[kVisited] += P_(kPartVisited, i);
        }
        if (i < n_levels) {
            acc[kCloses] += P_(kPartLvCloses, i);
            acc[kJoins] += P_(kPartLvJoins, i);
            acc[kVisited] += P_(kPartLvVisited, i);
        }
        if (i < n_live_edges) acc[kLiveE] += P_(kPartLiveEdges, i);
        if (i < n_qhw) {
            const uint64_t h = P_(kPartQhw, i);
            acc[kQhw] = h > acc[kQhw] ? h : acc[kQhw];
        }
    }
    const int w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
#pragma unroll
    for (int q = 0; q < kN; ++q) {
        uint64_t x = acc[q];
        if (q == kQhw) {
            for (int off = 32; off > 0; off >>= 1) {
                const uint64_t y = ((uint64_t)__shfl_xor((unsigned)(x >> 32), off) << 32) |
                                   __shfl_xor((unsigned)x, off);
                x = y > x ? y : x;
            }
        } else {
            x = wave_sum(x);
        }
        if (lane_id() == 0) red[q][w] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t tot[kN] = {};
        for (int q = 0; q < kN; ++q)
            for (int i = 0; i < nw; ++i)
                tot[q] = q == kQhw ? (red[q][i] > tot[q] ? red[q][i] : tot[q]) : tot[q] + red[q][i];
        stats->edges_total = tot[kEdges];
        stats->n_live = tot[kLive];
        stats->n_dead = (uint64_t)n - tot[kLive];
        stats->queued = (uint64_t)ctr[kQTail];
        stats->edges_sweep = tot[kSweep];
        stats->closes = tot[kCloses];
        stats->joins = tot[kJoins];
        stats->visited = tot[kVisited];
        stats->graph_edges = tot[kDeg];
        stats->q_highwater = tot[kQhw];
        stats->edges_live = tot[kLiveE];
        stats->stalled = ld_dev(ctr + kStall) != 0;
        stats->forest = (uint64_t)ld_dev(ctr + kJKilled);
        stats->jump_rounds = (uint64_t)ld_dev(ctr + kJRounds);
        stats->work_items = (uint64_t)(uint32_t)ld_dev(ctr + kJWork) +
                            (uint64_t)(uint32_t)ld_dev(ctr + kAcWork);
        stats->phases = (uint64_t)ld_dev(ctr + kLvPhases);
        stats->rechecks = ld_dev(reinterpret_cast<const uint64_t*>(ctr + kHyWork));
        if (ld_dev(ctr + kHyRounds)) stats->rounds = (uint64_t)ld_dev(ctr + kHyRounds);
        if (n == 0 && empty_rounds) stats->rounds = (uint64_t)empty_rounds;
    }
}

}  // namespace

}  // namespace trim
