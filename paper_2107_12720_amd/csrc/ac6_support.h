// ac6_support.h -- the AC-6 support search shared by the one-sided and the
// two-sided propagation (Section 6.1, DoPost): resume a vertex's scan from its
// cursor and join the list of the first live neighbour found.
#pragma once
#include "trim_device.h"

namespace trim {

// Split S_more lists: with `ext` (kMoreLists - 1 ints per vertex), S_more(w)
// is kMoreLists lists -- head[2w] and ext[(kMoreLists - 1) w ..] -- and
// joiner u goes to the list its id hashes to, so a closed hub's supporters
// come back as that many chains, walked side by side.  The hash (the top
// bits of a multiplicative one) and not the low bits of u: on R-MAT graphs
// the low id bits follow the generator's quadrant choices, and u mod 4 put
// up to 459 of one hub's 1,282 supporters in one list where the hash puts
// about a quarter.  S_last(w) stays one list (head[2w+1]).  ext == nullptr:
// one list.
__device__ __forceinline__ int* join_slot(int* head, int* ext, int w, bool last, int u) {
    if (last) return head + 2 * w + 1;
    const int s = (int)(((uint32_t)u * 0x9E3779B1u) >> (32 - kMoreListsLog));
    return (s == 0 || !ext) ? head + 2 * w : ext + (kMoreLists - 1) * w + (s - 1);
}
// The heads of a closed vertex's lists: more[] (kEmpty = none), last.
struct ClosedLists {
    int more[kMoreLists];
    int last;
};
// Close x: exchange every list head of x with kDead (the exchanges are
// independent, so their round trips overlap).  Each list, on its own, is
// closed with the guarantee of the unsplit close: nobody joins it after its
// exchange, and every earlier joiner comes back in the returned chain.
template <int S = __HIP_MEMORY_SCOPE_AGENT>
__device__ __forceinline__ ClosedLists close_lists(int* head, int* ext, int x) {
    ClosedLists c;
    const int2 ab = xchg2_s<S>(head + 2 * x, kDead, kDead);
    c.more[0] = ab.x;
    c.last = ab.y;
#pragma unroll
    for (int j = 1; j < kMoreLists; ++j)
        c.more[j] = ext ? xchg_s<S>(ext + (kMoreLists - 1) * x + (j - 1), kDead) : kEmpty;
    return c;
}

// Resume DoPost of u from cursor position p0 of its list in `g` (successors,
// or predecessors when `g` views G^T).  Returns true if u joined the support
// list of the first live neighbour found; `edges` receives the positions
// checked.  S: memory scope of the record store and the join (agent scope
// unless one workgroup owns the whole graph).  ext: the split S_more lists,
// or nullptr.
template <class View, int S = __HIP_MEMORY_SCOPE_AGENT>
__device__ __forceinline__ bool resume(const View& g, int u, int p0, int* head, uint64_t* rec,
                                       uint64_t& edges, int sched, int* ext = nullptr) {
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
            if (p + j < e) h[j] = ld_cached(join_slot(head, ext, w[j], p + j + 1 == e, u));
#pragma unroll
        for (int j = 0; j < kScan; ++j) {
            if (p + j >= e) break;
            int* slot = join_slot(head, ext, w[j], p + j + 1 == e, u);
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
