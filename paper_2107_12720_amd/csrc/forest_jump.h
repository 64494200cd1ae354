// forest_jump.h -- the forest collapse of AC-6 (Section 6.2 support lists),
// shared by the one-sided kernels and the two-sided ones (Section 4.1).
//
// After the first sweep, a vertex whose out-support is its last successor is
// removed exactly when that support is: these links (jp) form a forest, and
// every tree whose root the sweep left without a live successor falls with
// it.  jp[v] is the support of a tree member, v itself for a root whose fate
// is open, and ~v (< 0) for a removed root.  The sweep lists every member and
// every removed root (the latter with kRootBit).
#pragma once
#include "trim_device.h"
#include "trim_internal.h"
#include "block_append.h"
#include "grid_barrier.h"

namespace trim {

namespace {

// Forest-collapse list entries: a vertex id, with this bit for the vertices the
// sweep left without a live successor (the removed roots).
constexpr uint32_t kRootBit = 0x80000000u;

// One launch of at most two workgroups per CU, all resident at once: round r
// reads the list of round r (sizes rotate over three counters, like the AC-3
// lists), resolves what it can, appends the members still without a root to
// the list of round r + 1, and a grid barrier ends the round.  The links are
// updated in place; every value a later round reads (links, lists) is written
// and read with device-coherent accesses, so it is visible across XCDs after
// the barrier.  Stop rule: the unresolved member nearest its root always
// resolves in the next round (its link points at a resolved vertex or a
// root), so a round that resolves nothing leaves only members whose links run
// into a cycle.
// Entries per thread per step: more would leave most workgroups idle when a
// round's list is short.
constexpr int kJumpUnroll = 2;
// Links an entry follows per round (at least 2): a link that spans d levels
// spans kJumpHops * d after the round (2 is classic pointer doubling).
constexpr int kJumpHops = 8;
// Work items a removed vertex may hand back (its lists that are not members of
// its own tree): its S_more lists, plus the two in-side lists of the
// two-sided kernels.
constexpr int kJumpItems = kMoreLists + 2;

// Items of one round step buffered in LDS: up to kJumpItems per removed vertex,
// kJumpUnroll vertices per thread, plus what is left from before.
constexpr int kJumpStep = 256 * kJumpUnroll * kJumpItems;
constexpr int kJumpBuf = kJumpStep + 4096;

// Kill: `void operator()(int v, uint32_t (&item)[kJumpItems]) const` removes v
// (closes its lists) and fills the work items that hand its lists back, kNone
// for the unused ones.  v's out-side S_last list holds only members of v's
// own tree, which the same rounds remove, so Kill leaves it unwalked.
template <class Kill>
__global__ __launch_bounds__(256) void ac6_jump(Kill kill, int* jp, uint32_t* l0, uint32_t* l1,
                                                uint32_t* q, int* ctr, int max_rounds,
                                                int budget) {
    __shared__ uint32_t buf[kJumpBuf];   // hand-back items of removed vertices
    __shared__ int s_nbuf, s_base, s_wave[256 / kWave];
    __shared__ uint64_t red[16];
    if (ld_dev(ctr + kHyStop)) return;   // AC-6 rounds reached the fixed point
    if (threadIdx.x == 0) s_nbuf = 0;
    __syncthreads();
    auto flush = [&]() {
        __syncthreads();
        const int k = s_nbuf;
        if (k > 0) {
            if (threadIdx.x == 0) {
                add_dev(ctr + kPending, k);
                s_base = add_dev(ctr + kQTail, k);
            }
            __syncthreads();
            for (int i = threadIdx.x; i < k; i += blockDim.x) q[s_base + i] = buf[i];
            __syncthreads();
            if (threadIdx.x == 0) s_nbuf = 0;
        }
        __syncthreads();
    };
    uint64_t killed = 0;
    for (int r = 0; r < max_rounds; ++r) {
        const uint32_t* lin = (r & 1) ? l1 : l0;
        uint32_t* lout = (r & 1) ? l0 : l1;
        const int cnt = ld_dev(ctr + kJCnt0 + r % 3);
        if (cnt == 0 || (r > 0 && ld_dev(ctr + kJDone0 + (r - 1) % 3) == 0)) break;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st_dev(ctr + kJCnt0 + (r + 2) % 3, 0);
            st_dev(ctr + kJDone0 + (r + 1) % 3, 0);
            add_dev(ctr + kJRounds, 1);
            add_dev(ctr + kJWork, cnt);
        }
        uint64_t done = 0;
        const int step = gridDim.x * blockDim.x * kJumpUnroll;
        for (int base = blockIdx.x * blockDim.x * kJumpUnroll; base < cnt; base += step) {
            // anc[k][h]: where v[k]'s link leads after h + 1 links
            int v[kJumpUnroll], anc[kJumpUnroll][kJumpHops];
            uint32_t ent[kJumpUnroll];
#pragma unroll
            for (int k = 0; k < kJumpUnroll; ++k) {
                const int i = base + k * blockDim.x + threadIdx.x;
                ent[k] = i < cnt ? (uint32_t)ld_dev((const int*)lin + i) : kNone;
            }
#pragma unroll
            for (int k = 0; k < kJumpUnroll; ++k) {
                v[k] = (int)(ent[k] & ~kRootBit);
                anc[k][0] = (ent[k] != kNone && !(ent[k] & kRootBit)) ? ld_dev(jp + v[k]) : -1;
            }
            // further links, each one more dependent load; a link is followed
            // only from a member (a root's link is itself or < 0)
#pragma unroll
            for (int h = 1; h < kJumpHops; ++h)
#pragma unroll
                for (int k = 0; k < kJumpUnroll; ++k) {
                    const int a = anc[k][h - 1];
                    const bool member = a >= 0 && (h < 2 || a != anc[k][h - 2]);
                    anc[k][h] = member ? ld_dev(jp + a) : a;
                }
            int c = 0;
            uint32_t item[kJumpUnroll][kJumpItems];
            bool keep[kJumpUnroll];
#pragma unroll
            for (int k = 0; k < kJumpUnroll; ++k) {
#pragma unroll
                for (int j = 0; j < kJumpItems; ++j) item[k][j] = kNone;
                keep[k] = false;
                bool dies = false;
                if (ent[k] == kNone) {
                    // past the end of the list
                } else if (ent[k] & kRootBit) {
                    dies = true;                 // a removed root
                } else {
                    // the first link that is a removed root's mark (< 0) or an
                    // open root (its link is itself) settles v; else v keeps
                    // the farthest ancestor
                    int prev = anc[k][0], outcome = 0, to = anc[k][kJumpHops - 1];
#pragma unroll
                    for (int h = 1; h < kJumpHops; ++h) {
                        const int a = anc[k][h];
                        if (outcome == 0 && a < 0) {
                            outcome = 1;
                            to = a;
                        } else if (outcome == 0 && a == prev) {
                            outcome = 2;
                            to = prev;
                        }
                        prev = a;
                    }
                    if (outcome == 1) {          // the root is removed, so v is
                        st_dev(jp + v[k], to);
                        dies = true;
                        done += 1;
                    } else if (outcome == 2) {   // the root's fate is open
                        if (to != anc[k][0]) st_dev(jp + v[k], to);
                        done += 1;
                    } else {
                        st_dev(jp + v[k], to);
                        keep[k] = true;
                        c += 1;
                    }
                }
                if (dies) {
                    kill(v[k], item[k]);
                    killed += 1;
                }
            }
            int slot = block_append_base(c, ctr + kJCnt0 + (r + 1) % 3, nullptr, s_wave, &s_base);
#pragma unroll
            for (int k = 0; k < kJumpUnroll; ++k) {
                if (keep[k]) st_dev((int*)lout + slot++, v[k]);
#pragma unroll
                for (int j = 0; j < kJumpItems; ++j) {
                    const uint64_t mask = ballot(item[k][j] != kNone);
                    if (mask) {
                        int wbase = 0;
                        if (lane_id() == 0) wbase = atomicAdd(&s_nbuf, popc(mask));
                        wbase = __shfl(wbase, 0);
                        if (item[k][j] != kNone)
                            buf[wbase + popc(mask & lanes_below())] = item[k][j];
                    }
                }
            }
            __syncthreads();
            if (s_nbuf > kJumpBuf - kJumpStep) flush();
        }
        done = block_sum(done, red);
        if (threadIdx.x == 0 && done) add_dev(ctr + kJDone0 + r % 3, (int)done);
        if (!grid_barrier(ctr + kBarCount, ctr + kBarGen, ctr + kStall, budget)) break;
    }
    flush();
    killed = block_sum(killed, red);
    if (threadIdx.x == 0 && killed) add_dev(ctr + kJKilled, (int)killed);
}

constexpr int kLevelsPerCu = 2;
// Workgroups of the level-synchronous launches (propagation phases and forest
// rounds): two per CU, fewer for small graphs, where a phase holds few items
// and the grid barrier, whose cost grows with the number of arriving
// workgroups, dominates (one workgroup per 4,096 vertices, at least 8).
__host__ inline int phase_blocks(long long n, int cus) {
    long long b = n / 4096;
    if (b < 8) b = 8;
    if (b > (long long)cus * kLevelsPerCu) b = (long long)cus * kLevelsPerCu;
    return (int)b;
}

// Rounds that resolve any depth: ceil(log2 n) + 1 (each round at least
// doubles the span of every unresolved link).
inline int jump_rounds(int n) {
    int rounds = 2;
    while ((1LL << (rounds - 1)) < (long long)n) ++rounds;
    return rounds;
}

}  // namespace

}  // namespace trim
