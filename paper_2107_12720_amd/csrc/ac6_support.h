// ac6_support.h -- the AC-6 support search shared by the one-sided and the
// two-sided propagation (Section 6.1, DoPost): resume a vertex's scan from its
// cursor and join the list of the first live neighbour found.
#pragma once
#include "trim_device.h"

namespace trim {

// Resume DoPost of u from cursor position p0 of its list in `g` (successors,
// or predecessors when `g` views G^T).  Returns true if u joined the support
// list of the first live neighbour found; `edges` receives the positions
// checked.  S: memory scope of the record store and the join (agent scope
// unless one workgroup owns the whole graph).
template <class View, int S = __HIP_MEMORY_SCOPE_AGENT>
__device__ __forceinline__ bool resume(const View& g, int u, int p0, int* head, uint64_t* rec,
                                       uint64_t& edges, int sched) {
    // kScan successors at a time: their targets, then their list heads, each
    // group of loads in flight together, then the joins in list order.
    constexpr int kScan = 4;
    const int e = g.end(u);
    const int ctx = g.vctx(u);
    for (int p = p0; p < e; p += kScan) {
        int w[kScan], h[kScan];
#pragma unroll
        for (int j = 0; j < kScan; ++j)
            if (p + j < e) w[j] = g.target(u, p + j, ctx);
#pragma unroll
        for (int j = 0; j < kScan; ++j)
            if (p + j < e) h[j] = ld_cached(head + 2 * w[j] + (p + j + 1 == e));
#pragma unroll
        for (int j = 0; j < kScan; ++j) {
            if (p + j >= e) break;
            int* slot = head + 2 * w[j] + (p + j + 1 == e);
            int hj = h[j];
            while (hj != kDead) {
                st_s<S>(rec + u, pack_rec(hj, p + j));
                complete_mem();
                if (sched & TRIM_SCHED_JITTER) jitter_nap(((uint64_t)u << 24) ^ (p + j));
                if (cas_s<S>(slot, hj, u)) {
                    edges += (uint64_t)(p + j - p0 + 1);
                    return true;
                }
            }
        }
    }
    edges += (uint64_t)(e - p0);
    return false;
}

}  // namespace trim
