// ac4.hip -- AC-4-based graph trimming on gfx950 (Section 5.2, Alg. par-ac4trim).
//
// cnt[v] is the live out-degree counter, initialised from CSR offsets
// (AC4Trim*, Section 9.3: no edge is traversed to find it).  A removed vertex
// w decrements cnt[u] once for every edge u -> w, walking w's predecessors in
// the transposed graph.  The paper takes CAS(status, LIVE, DEAD) to enqueue a
// vertex once; here the fetch-and-add that brings cnt[u] from 1 to 0 returns
// 1 to exactly one lane, which makes that lane u's unique remover, so the
// status is simply cnt[u] == 0.
//
// Two-sided (Section 4.1, the in-degree check over G^T): cnt[n+v] also counts
// v's live predecessors, from the G^T offsets.  A removed w then decrements
// the out-counters of its predecessors and the in-counters of its successors;
// a vertex can reach zero on both counters, so the lane that brings either to
// zero removes it only if its exchange of dead[v] is the first one.  Every
// removed vertex walks both of its lists once.
//
// Kernels: ac4_init (counters), ac4_seed (out-degree-0 vertices queued),
// ac4_propagate (persistent workers on per-wavefront LDS rings, WaveQueue;
// a lane walks a short predecessor list of its removed vertex eight at a
// time, with the eight decrements in flight together, and then goes on with
// one of the vertices it removed itself, depth first; long lists are walked
// by the whole wavefront), ac4_pack (bitmap from cnt > 0).
#include "trim_device.h"
#include "trim_stats.h"
#include "trim_internal.h"
#include "block_append.h"

namespace trim {

namespace {

// A preset vertex (removed before trimming) starts at cnt = 0: it is queued
// like an out-degree-0 vertex, and its counter only goes negative after that,
// so no decrement ever returns 1 for it.
template <bool kTwo>
__global__ void ac4_init(const int* row_off, const int* rrow_off, const uint32_t* preset, int n,
                         int* cnt, int* dead, int* ctr, uint64_t* worker_edges, int P,
                         trim_stats_t* stats) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < kCtrInts) ctr[tid] = 0;
    for (int p = tid; p < P; p += gridDim.x * blockDim.x) worker_edges[p] = 0;
    if (stats && tid < (int)(sizeof(trim_stats_t) / 8)) ((uint64_t*)stats)[tid] = 0;
    for (int v = tid; v < n; v += gridDim.x * blockDim.x) {
        const int d = row_off[v + 1] - row_off[v];
        cnt[v] = (preset && ((preset[v >> 5] >> (v & 31)) & 1u)) ? 0 : d;
        if (kTwo) {
            const int di = rrow_off[v + 1] - rrow_off[v];
            cnt[n + v] = di;
            dead[v] = (d == 0 || di == 0) ? 1 : 0;
        }
    }
}

// Four vertices per thread, one shared-queue reservation per block and step.
template <bool kTwo>
__global__ void ac4_seed(const int* cnt, const int* dead, int n, uint32_t* q, int* ctr) {
    __shared__ int s_wave[1024 / kWave], s_base;
    const int step = gridDim.x * blockDim.x * 4;
    for (int base = blockIdx.x * blockDim.x * 4; base < n; base += step) {
        int v[4], c = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = base + j * blockDim.x + threadIdx.x;
            const bool d = x < n && (kTwo ? dead[x] != 0 : cnt[x] == 0);
            v[j] = d ? x : -1;
            c += d;
        }
        int slot = block_append_base(c, ctr + kQTail, ctr + kPending, s_wave, &s_base);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (v[j] >= 0) q[slot++] = make_item(0, v[j]);
    }
}

// The lane whose decrement brought a counter of u to zero: u's remover?
template <bool kTwo>
__device__ __forceinline__ bool removes(int* dead, int u) {
    return !kTwo || xchg_dev(dead + u, 1) == 0;
}

constexpr int kBatch = 8;
constexpr int kCoop = 16;   // predecessor lists longer than this are walked by the wavefront
// Busy iterations between polls for waiting lanes elsewhere: 16, as for the
// AC-6 kernels on explicit graphs (measured at 512 workers: the 65,536-vertex
// core+tail graph 35 % and R-MAT 22 with half of its vertices preset 12 %
// faster than with 64, the R-MAT 22 chain workload unchanged).
constexpr int kShareEvery4 = 16;

// Phase 0 walks pre(w) over G^T and decrements out-counters (cnt[u]); with
// kTwo, phase 1 then walks post(w) over G and decrements in-counters
// (cnt[n + x]).
template <bool kTwo>
__global__ __launch_bounds__(256) void ac4_propagate(const int* rrow_off, const int* rcol,
                                                     const int* row_off, const int* col, int n,
                                                     int* cnt, int* dead, uint32_t* q, int* ctr,
                                                     uint64_t* worker_edges, uint64_t* part,
                                                     int sched, int budget) {
    __shared__ uint32_t rings[256 / kWave][kLocalQ];
    __shared__ int ring_tail[256 / kWave];
    WaveQueue wq;
    const int wv = threadIdx.x / kWave;
    wq.init(rings[wv], &ring_tail[wv], q, ctr + kQHead, ctr + kQTail, ctr + kPending,
            ctr + kStall, budget, kShareEvery4);
    uint32_t item = kNone;
    int k = 0, e = 0, ph = 0;
    bool started = false;
    uint64_t edges = 0;
    while (wq.acquire(item)) {
        uint32_t out[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) out[j] = kNone;
        if (item != kNone && !started) {
            const int w = item_vertex(item);
            k = rrow_off[w];
            e = rrow_off[w + 1];
            ph = 0;
            started = true;
            edges += (uint64_t)(e - k);
            if (kTwo) edges += (uint64_t)(row_off[w + 1] - row_off[w]);
        }
        // Long predecessor lists: the whole wavefront walks them, one list at
        // a time, 64 x kBatch decrements in flight per round.
        for (uint64_t big = ballot(item != kNone && e - k > kCoop); big; big &= big - 1) {
            const int owner = __ffsll((unsigned long long)big) - 1;
            const int kb = __shfl(k, owner), eb = __shfl(e, owner);
            const int phb = kTwo ? __shfl(ph, owner) : 0;
            const int* adj = phb ? col : rcol;
            int* ctr_of = phb ? cnt + n : cnt;
            for (int base = kb; base < eb; base += kWave * kBatch) {
                int u[kBatch], old[kBatch];
                uint32_t o[kBatch];
#pragma unroll
                for (int j = 0; j < kBatch; ++j) {
                    const int p = base + j * kWave + lane_id();
                    if (p < eb) u[j] = adj[p];
                }
                if (sched & TRIM_SCHED_JITTER) jitter_nap(((uint64_t)kb << 20) ^ base);
#pragma unroll
                for (int j = 0; j < kBatch; ++j) {
                    const int p = base + j * kWave + lane_id();
                    if (p < eb) old[j] = add_dev(ctr_of + u[j], -1);
                }
#pragma unroll
                for (int j = 0; j < kBatch; ++j) {
                    const int p = base + j * kWave + lane_id();
                    o[j] = (p < eb && old[j] == 1 && removes<kTwo>(dead, u[j])) ? make_item(0, u[j])
                                                                               : kNone;
                }
#pragma unroll
                for (int j = 0; j < kBatch; j += 2) wq.push(o[j], o[j + 1]);
            }
            if (lane_id() == owner) {
                if (kTwo && ph == 0) {   // on to the successors of the owner's vertex
                    const int w = item_vertex(item);
                    k = row_off[w];
                    e = row_off[w + 1];
                    ph = 1;
                } else {
                    item = kNone;
                    started = false;
                }
            }
        }
        if (item != kNone) {
            const int nb = min(kBatch, e - k);
            const int* adj = (kTwo && ph) ? col : rcol;
            int* ctr_of = (kTwo && ph) ? cnt + n : cnt;
            int u[kBatch], old[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                if (j < nb) u[j] = adj[k + j];
            if (sched & TRIM_SCHED_JITTER) jitter_nap(((uint64_t)k << 16) ^ item);
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                if (j < nb) old[j] = add_dev(ctr_of + u[j], -1);
#pragma unroll
            for (int j = 0; j < kBatch; ++j)   // u's last live neighbour on this side
                if (j < nb && old[j] == 1 && removes<kTwo>(dead, u[j])) out[j] = make_item(0, u[j]);
            k += nb;
            if (kTwo && k >= e && ph == 0) {   // on to the successors
                const int w = item_vertex(item);
                k = row_off[w];
                e = row_off[w + 1];
                ph = 1;
            }
            if (k >= e) {
                item = kNone;
                started = false;
                // depth first: go on with one vertex this lane has just
                // removed instead of handing it to the queue
#pragma unroll
                for (int j = 0; j < kBatch; ++j)
                    if (item == kNone && out[j] != kNone) {
                        item = out[j];
                        out[j] = kNone;
                    }
            }
        }
#pragma unroll
        for (int j = 0; j < kBatch; j += 2) wq.push(out[j], out[j + 1]);
        wq.rebalance();
    }
    edges = wave_sum(edges);
    if (lane_id() == 0 && edges) add_dev(worker_edges + blockIdx.x, edges);
    __shared__ int red[16];
    const int qhw = block_max(wq.hw, red);
    if (threadIdx.x == 0) part[kPartQhw * kPartStride + blockIdx.x] = (uint64_t)qhw;
}

struct Ac4Live {
    const int* cnt;
    __device__ __forceinline__ bool operator()(int v) const { return cnt[v] > 0; }
};
struct Ac4TwoLive {
    const int* dead;
    __device__ __forceinline__ bool operator()(int v) const { return dead[v] == 0; }
};

inline int grid_for(long long n, int block, int max_blocks = 1 << 20) {
    long long b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

template <bool kTwo>
hipError_t ac4_run(const trim_csr_t& g, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                   uint64_t* worker_edges, trim_stats_t* stats, const uint32_t* preset) {
    const int n = g.n, P = lc.workers, B = lc.block;
    int pack_blocks = 0;
    {
        Timed t(lc, kTwo ? "ac4t_init" : "ac4_init");
        hipLaunchKernelGGL(ac4_init<kTwo>, dim3(grid_for(n, 256, 16384)), dim3(256), 0,
                           lc.stream, g.row_off, g.rrow_off, preset, n, w.a, w.d, w.ctr,
                           worker_edges, P, stats);
    }
    if (n > 0) {
        {
            Timed t(lc, kTwo ? "ac4t_seed" : "ac4_seed");
            hipLaunchKernelGGL(ac4_seed<kTwo>, dim3(grid_for(n, 4 * B, lc.cus * 8)), dim3(B), 0,
                               lc.stream, w.a, w.d, n, w.q, w.ctr);
        }
        {
            Timed t(lc, kTwo ? "ac4t_propagate" : "ac4_propagate");
            hipLaunchKernelGGL(ac4_propagate<kTwo>, dim3(P), dim3(256), 0, lc.stream, g.rrow_off,
                               g.rcol, g.row_off, g.col, n, w.a, w.d, w.q, w.ctr, worker_edges,
                               w.part, lc.schedule, lc.budget);
        }
        Timed t(lc, kTwo ? "ac4t_pack" : "ac4_pack");
        pack_blocks = grid_for(n, 256, lc.cus * 4);
        if (kTwo)
            hipLaunchKernelGGL(pack_bitmap<Ac4TwoLive>, dim3(pack_blocks), dim3(256), 0, lc.stream,
                               Ac4TwoLive{w.d}, n, bitmap, w.part, w.ctr, w.q, w.qwords);
        else
            hipLaunchKernelGGL(pack_bitmap<Ac4Live>, dim3(pack_blocks), dim3(256), 0, lc.stream,
                               Ac4Live{w.a}, n, bitmap, w.part, w.ctr, w.q, w.qwords);
    }
    if (stats)
        hipLaunchKernelGGL(finalize_stats, dim3(1), dim3(1024), 0, lc.stream, n, P, 0, 0,
                           pack_blocks, n > 0 ? P : 0, worker_edges, w.part, w.ctr, stats, 0);
    return hipGetLastError();
}

}  // namespace

hipError_t ac4_csr(const trim_csr_t& g, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                   uint64_t* worker_edges, trim_stats_t* stats, const uint32_t* preset) {
    return ac4_run<false>(g, w, lc, bitmap, worker_edges, stats, preset);
}

hipError_t ac4_two_csr(const trim_csr_t& g, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                       uint64_t* worker_edges, trim_stats_t* stats) {
    return ac4_run<true>(g, w, lc, bitmap, worker_edges, stats, nullptr);
}

int ac4_max_workers_per_cu(int) {
    int nb = 0, nb2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ac4_propagate<false>, 256, 0) !=
        hipSuccess)
        return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, ac4_propagate<true>, 256, 0) ==
            hipSuccess &&
        nb2 < nb)
        nb = nb2;
    return nb < 1 ? 1 : nb;
}

}  // namespace trim
