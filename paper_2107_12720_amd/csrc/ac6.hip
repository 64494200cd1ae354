// ac6.hip -- AC-6-based graph trimming on gfx950 (Section 6.2, Alg. par-ac-6-trim).
//
// State per vertex v:
//   head[2v], head[2v+1]  the supporting set S(v) (Def. Supporting Set), split
//            in two intrusive linked lists: S_more(v) holds supporters with
//            successors left after v, S_last(v) those for which v is the last
//            successor.  Each head is kEmpty, the id of the last vertex that
//            joined, or kDead once v is removed; kDead closes the list.
//   rec[v]   (next, cursor): the next member of the list v is in, and the
//            position of v's current support in its successor list.
//
// The split matters for depth: when v is removed, every member of S_last(v)
// is removed too, with no successor left to check.  The closer learns the
// first of them from its own exchange and closes it at once, so each step of
// a peeling chain costs one atomic round trip instead of a list walk plus a
// record load.
//
// The paper's Lock(w)/recheck/add and Lock(v)/DEAD/Unlock become lock-free:
//   join   : rec[v] = (h, p); CAS(head[w], h, v)  -- fails once head[w] == kDead
//   close  : one 8-byte exchange of both heads of v with kDead -- takes both
//            lists whole at once
// which gives the guarantee of the locks: after the close nobody joins S(v),
// and everybody who joined before it is handed back exactly once.  Lanes of a
// wavefront run in lock step, so a spinning lock would deadlock there.
//
// A vertex that finds no live successor is not closed on the spot: it becomes
// a "close item".  Vertices may still join it until it is closed; the closer
// hands them back, so they simply move on to their next successor (the edge
// was checked once).  Every successor position is passed at most once, so the
// number of successor checks is the same for every schedule:
//   sum_dead deg(v) + sum_live (first-live-successor index + 1).
//
// Kernels, in stream order:
//   ac6_init       heads = kDead for out-degree-0 vertices (their lists are
//                  empty, nothing to hand back) and for vertices removed
//                  before trimming (the optional preset bitmap: the vertex
//                  sampling of Section 9), kEmpty otherwise; the sinks bitmap
//                  marks both; counters and outputs zeroed.
//   ac6_sweep      DoPost for every vertex, one lane per vertex.  Only sinks
//                  are removed while this kernel runs, so a target is live iff
//                  its sinks bit is clear, and joining is a plain exchange (no
//                  CAS retry storms on hub vertices).  Vertices without a live
//                  successor are queued as close items.
//   ac6_jump       (forest collapse, the default) after the sweep, a vertex
//                  whose support is its last successor is removed exactly
//                  when that support is: these links form a forest, and every
//                  tree whose root the sweep left without a live successor is
//                  removed at once.  Pointer jumping over the tree members
//                  (rounds in one launch, links updated in place; a round
//                  follows kJumpHops links, so after r rounds a link spans
//                  kJumpHops^r levels: O(log depth) rounds)
//                  finds each member's root; a member whose root is removed
//                  is removed (both heads exchanged with kDead) and its S_more
//                  list handed to the propagation.  Its S_last list holds only
//                  members of its own tree, removed by the same rounds, so it
//                  is not walked.  No successor is checked here.  A round in
//                  which no member found its root leaves only members whose
//                  links run into a cycle: they stay live, and the rounds stop.
//   ac6_propagate  persistent workers (the paper's Trim_p) run close and walk
//                  items (see below) through per-wavefront LDS rings
//                  (WaveQueue); a lane follows an S_last chain for up to
//                  kHops removals in a row.  Exits when no item is pending.
//   ac6_pack       live bitmap by wavefront ballot, live/dead counts.
#include "trim_device.h"
#include "trim_stats.h"
#include "trim_internal.h"
#include "ac6_support.h"
#include "block_append.h"
#include "grid_barrier.h"
#include "forest_jump.h"

namespace trim {

namespace {

// Table staging: the implicit view reads its degree thresholds from LDS.
template <class View>
struct Stage {
    static constexpr int kWords = 1;
    __device__ static void apply(View&, uint64_t*) {}
};
template <>
struct Stage<ImplicitView> {
    static constexpr int kWords = 256;
    __device__ static void apply(ImplicitView& g, uint64_t* lds) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) lds[i] = g.table[i];
        __syncthreads();
        g.table = lds;
    }
};

// Busy iterations of a propagation wavefront between polls for waiting lanes
// elsewhere (WaveQueue::rebalance), chosen per view by measurement at the
// default 512 workers: polling every 16 instead of 64 iterations made the
// propagation of the 4,096-graph batch about 25 % and of the 65,536-vertex
// core+tail graph about 40 % faster, left the R-MAT 22 chain workload
// unchanged, and made the implicit 2^28 graph's propagation about 25 % slower.
template <class View>
struct ShareEvery {
    static constexpr int value = 16;
};
template <>
struct ShareEvery<ImplicitView> {
    static constexpr int value = 64;
};

// A filter of the removals of one round: 2^log2 bits, vertex v at a
// multiplicative hash of its id (R-MAT ids carry the generator's quadrant
// choices in their low bits), three slots used in rotation (see ac6_round).
struct RoundFilter {
    uint32_t* f = nullptr;   // 3 slots of 2^(log2 - 5) words
    int log2 = 5;
    __device__ __forceinline__ int words() const { return 1 << (log2 - 5); }
    __device__ __forceinline__ uint32_t* slot(int r) const { return f + (r % 3) * words(); }
    __device__ __forceinline__ uint32_t hash(int v) const {
        return ((uint32_t)v * 0x9E3779B1u) >> (32 - log2);
    }
    __device__ __forceinline__ void add(int r, int v) const {
        const uint32_t h = hash(v);
        atomicOr(slot(r) + (h >> 5), 1u << (h & 31));
    }
};

// Also writes sinks[]: bit v set iff v has no successor or is preset.  During
// the first sweep these are the only removed vertices, so the sweep tests this
// small, cache-resident bitmap instead of a list head in HBM.  Each wavefront
// covers 64 consecutive ids (blockDim and the grid stride are multiples of
// 64); the last wavefront may write one word past ceil(n/32), which the
// buffer has.
//
// With late support registration (opts.rounds >= 2, sinks2 != NULL) the heads
// are left for ac6_heads, and the bitmap is written twice: the round bitmaps
// start equal (see ac6_round).
template <class View>
__global__ void ac6_init(View g, int n, int* head, int* ext, uint32_t* sinks, uint32_t* sinks2,
                         const uint32_t* preset, int* ctr, uint64_t* worker_edges, int P,
                         trim_stats_t* stats, RoundFilter flt) {
    __shared__ uint64_t lds[Stage<View>::kWords];
    Stage<View>::apply(g, lds);
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < kCtrInts) ctr[tid] = (tid == kHyRounds && sinks2) ? 1 : 0;
    // the filter slots rounds 1 and 2 write
    if (flt.f)
        for (int i = tid; i < 2 * flt.words(); i += gridDim.x * blockDim.x)
            flt.slot(1)[i] = 0;
    for (int p = tid; p < P; p += gridDim.x * blockDim.x) worker_edges[p] = 0;
    if (stats && tid < (int)(sizeof(trim_stats_t) / 8)) ((uint64_t*)stats)[tid] = 0;
    for (int v = tid; v < n; v += gridDim.x * blockDim.x) {
        const bool sink =
            g.end(v) == g.begin(v) || (preset && ((preset[v >> 5] >> (v & 31)) & 1u));
        const int h = sink ? kDead : kEmpty;
        if (head) {
            reinterpret_cast<int2*>(head)[v] = make_int2(h, h);
            if (ext)
                for (int j = 0; j < kMoreLists - 1; ++j)
                    ext[(kMoreLists - 1) * (long long)v + j] = h;
        }
        const uint64_t m = ballot(sink);
        if (lane_id() == 0) {
            sinks[v >> 5] = (uint32_t)m;
            sinks[(v >> 5) + 1] = (uint32_t)(m >> 32);
            if (sinks2) {
                sinks2[v >> 5] = (uint32_t)m;
                sinks2[(v >> 5) + 1] = (uint32_t)(m >> 32);
            }
        }
    }
}

// The init of late registration on an explicit graph: no list heads, only
// the two round bitmaps of the sinks.  A lane takes four consecutive vertices
// from one 16-byte load of the offsets (and the next offset), a wavefront 256
// vertices, whose eight bitmap words it assembles by shuffles.  Offsets that
// are not 16-byte aligned take the one-vertex-per-lane path of ac6_init.
__global__ void ac6_init_bits(const int* row_off, int n, uint32_t* y1, uint32_t* y0, int* ctr,
                              uint64_t* worker_edges, int P, trim_stats_t* stats,
                              RoundFilter flt) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    if (tid < kCtrInts) ctr[tid] = tid == kHyRounds ? 1 : 0;
    for (int p = tid; p < P; p += stride) worker_edges[p] = 0;
    if (stats && tid < (int)(sizeof(trim_stats_t) / 8)) ((uint64_t*)stats)[tid] = 0;
    if (flt.f)
        for (int i = tid; i < 2 * flt.words(); i += stride) flt.slot(1)[i] = 0;
    const int ngroups = (n + 3) >> 2;   // groups of four vertices
    const int nwords = (n + 31) >> 5;
    const int lane = lane_id();
    const int waves = stride / kWave;
    for (int g0 = (tid / kWave) * kWave; g0 < ngroups; g0 += waves * kWave) {
        const int gi = g0 + lane;
        uint32_t nib = 0;
        if (gi < ngroups) {
            const int v = gi << 2;
            if (v + 4 <= n) {
                typedef int v4i __attribute__((ext_vector_type(4)));
                const v4i a = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(row_off) + gi);
                const int e4 = __builtin_nontemporal_load(row_off + v + 4);
                nib = (uint32_t)(a.x == a.y) | ((uint32_t)(a.y == a.z) << 1) |
                      ((uint32_t)(a.z == a.w) << 2) | ((uint32_t)(a.w == e4) << 3);
            } else {
                for (int j = 0; v + j < n; ++j)
                    nib |= (uint32_t)(row_off[v + j] == row_off[v + j + 1]) << j;
            }
        }
        // word (g0 / 8 + lane / 8) holds the nibbles of lanes 8k .. 8k + 7
        uint32_t word = nib << (4 * (lane & 7));
        word |= __shfl_xor(word, 1);
        word |= __shfl_xor(word, 2);
        word |= __shfl_xor(word, 4);
        const int wi = (g0 >> 3) + (lane >> 3);
        if ((lane & 7) == 0 && wi < nwords) {
            y1[wi] = word;
            y0[wi] = word;
        }
    }
}

constexpr int kCasBuf = 4096;   // entries buffered in LDS before one shared-queue append
constexpr int kSweepUnroll = 4; // vertices per lane in flight in the first sweep
constexpr int kSweepUnrollDefer = 8;   // the same without joins (late registration)
// Round-list entries (late support registration): (vertex, cursor target)
// with flag bits on the target: the cursor is at the vertex's last successor;
// the vertex was removed by a round (the entry is skipped from then on); the
// cursor is still at the vertex's first successor (else it is in cur[v]).
constexpr uint32_t kLastBit = 0x80000000u;
constexpr uint32_t kGoneBit = 0x40000000u;
constexpr uint32_t kFirstBit = 0x20000000u;
constexpr uint32_t kTargetMask = 0x1FFFFFFFu;


// With jp (the forest collapse): jp[v] = the target of v's support if that is
// v's last successor (v is a tree member, listed in jlist), v itself if v has
// successors left after its support (a root whose fate is open), and ~v (< 0)
// if v has no live successor (a removed root, listed with kRootBit).  Without
// jp, the vertices without a live successor are queued as close items.
//
// Each lane keeps kSweepUnroll vertices in flight, blockDim apart (so every
// load of a step is coalesced across the wavefront): the offsets of all of
// them, then their first targets and those targets' sinks bits, then their
// joins, are issued before any result is waited for.  The first successor is
// almost always the support (a sink is rarely anyone's first target), so the
// serial scan past sinks is the exception.  The join's exchange returns the
// old head, which goes into the joiner's record: with several joins in flight
// their round trips overlap instead of adding up.
//
// kDefer (late support registration, the first of opts.rounds rounds): no
// vertex joins a list.  A vertex with a live successor is appended to the
// round-2 list with its cursor (see ac6_round); one without becomes a removal
// of round 1, set in the round bitmap `ynext` and counted.
template <class View, bool kDefer>
__global__ void ac6_sweep(View g, int n, int chunk, int* head, int* ext, const uint32_t* sinks,
                          const uint32_t* preset, uint64_t* rec, uint32_t* q, int* ctr,
                          uint64_t* worker_edges, int P, uint64_t* part, int sched, int* jp,
                          uint32_t* jlist, uint32_t* ynext, int* lout, long long hcap,
                          int* cur, RoundFilter flt) {
    constexpr int U = kDefer ? kSweepUnrollDefer : kSweepUnroll;
    __shared__ uint64_t lds[Stage<View>::kWords];
    __shared__ uint32_t cas[kDefer ? 1 : kCasBuf];
    __shared__ int s_chunk, s_ncas, s_base, s_wave[1024 / kWave];
    __shared__ uint64_t red[16];
    Stage<View>::apply(g, lds);
    if (threadIdx.x == 0) s_ncas = 0;
    uint64_t edges = 0, degsum = 0, removed = 0;
    // move the buffered entries to the shared queue (close items) or to the
    // forest list, with one reservation
    auto flush = [&]() {
        __syncthreads();
        const int k = s_ncas;
        if (k > 0) {
            if (threadIdx.x == 0) {
                if (jp) {
                    s_base = add_dev(ctr + kJCnt0, k);
                } else {
                    add_dev(ctr + kPending, k);
                    s_base = add_dev(ctr + kQTail, k);
                }
            }
            __syncthreads();
            uint32_t* dst = jp ? jlist : q;
            for (int i = threadIdx.x; i < k; i += blockDim.x) dst[s_base + i] = cas[i];
            __syncthreads();
            if (threadIdx.x == 0) s_ncas = 0;
        }
        __syncthreads();
    };
    for (;;) {
        // claim the next chunk of vertices (schedule(dynamic, chunk))
        if (threadIdx.x == 0) s_chunk = add_dev(ctr + kCursor, chunk);
        __syncthreads();
        const int claim = s_chunk;
        __syncthreads();
        if (claim >= n) break;
        int cb = claim;
        if (sched & TRIM_SCHED_REVERSE) cb = ((n + chunk - 1) / chunk - 1 - claim / chunk) * chunk;
        const int ce = cb + chunk < n ? cb + chunk : n;
        for (int base = cb; base < ce; base += U * blockDim.x) {
            int v[U], b[U], e[U], gi[U], p[U], w[U];
            bool ok[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                v[k] = base + k * blockDim.x + threadIdx.x;
                b[k] = e[k] = 0;
                gi[k] = 0;
                if (v[k] < ce) {
                    b[k] = g.begin(v[k]);
                    e[k] = g.end(v[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                degsum += (uint64_t)(e[k] - b[k]);
                // a preset vertex is removed already: no DoPost
                if (preset && b[k] < e[k] && ((preset[v[k] >> 5] >> (v[k] & 31)) & 1u))
                    e[k] = b[k];
                p[k] = b[k];
                w[k] = 0;
                if (b[k] < e[k]) {
                    gi[k] = g.vctx(v[k]);
                    w[k] = g.target(v[k], b[k], gi[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                ok[k] = b[k] < e[k] && !((sinks[w[k] >> 5] >> (w[k] & 31)) & 1u);
            }
            // the rare serial scan past sinks
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (b[k] < e[k] && !ok[k]) {
                    for (++p[k]; p[k] < e[k]; ++p[k]) {
                        w[k] = g.target(v[k], p[k], gi[k]);
                        if (!((sinks[w[k] >> 5] >> (w[k] & 31)) & 1u)) break;
                    }
                    ok[k] = p[k] < e[k];
                }
            }
            if constexpr (kDefer) {
                int c = 0;
#pragma unroll
                for (int k = 0; k < U; ++k) c += ok[k];
                int slot = block_append_base(c, ctr + kHyCnt0, nullptr, s_wave, &s_base);
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    if (ok[k]) {
                        lout[slot] = v[k];
                        lout[hcap + slot] = (int)((uint32_t)w[k] |
                                                  (p[k] + 1 == e[k] ? kLastBit : 0u) |
                                                  (p[k] == b[k] ? kFirstBit : 0u));
                        if (p[k] != b[k]) cur[v[k]] = p[k];
                        ++slot;
                        edges += (uint64_t)(p[k] - b[k] + 1);
                    } else if (b[k] < e[k]) {
                        atomicOr(ynext + (v[k] >> 5), 1u << (v[k] & 31));
                        flt.add(1, v[k]);
                        removed += 1;
                        edges += (uint64_t)(e[k] - b[k]);
                    }
                }
                continue;
            }
            int old[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (ok[k]) {
                    if (sched & TRIM_SCHED_JITTER)
                        jitter_nap(((uint64_t)blockIdx.x << 32) ^ (uint32_t)v[k]);
                    old[k] = xchg_dev(join_slot(head, ext, w[k], p[k] + 1 == e[k], v[k]), v[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                bool casualty = false, member = false;
                if (ok[k]) {
                    rec[v[k]] = pack_rec(old[k], p[k]);
                    edges += (uint64_t)(p[k] - b[k] + 1);
                    if (jp) {
                        member = p[k] + 1 == e[k];
                        jp[v[k]] = member ? w[k] : v[k];
                    }
                } else if (b[k] < e[k]) {
                    casualty = true;
                    if (jp) jp[v[k]] = ~v[k];
                    edges += (uint64_t)(e[k] - b[k]);
                }
                const bool put = casualty || member;
                const uint64_t mask = ballot(put);
                if (mask) {
                    int wbase = 0;
                    if (lane_id() == 0) wbase = atomicAdd(&s_ncas, popc(mask));
                    wbase = __shfl(wbase, 0);
                    if (put)
                        cas[wbase + popc(mask & lanes_below())] =
                            jp ? ((uint32_t)v[k] | (casualty ? kRootBit : 0u))
                               : make_item(0, v[k]);
                }
            }
            __syncthreads();
            if (s_ncas > kCasBuf - U * (int)blockDim.x) flush();
        }
    }
    if constexpr (!kDefer) flush();
    edges = block_sum(edges, red);
    degsum = block_sum(degsum, red);
    if constexpr (kDefer) removed = block_sum(removed, red);
    if (threadIdx.x == 0) {
        if (edges) add_dev(worker_edges + (blockIdx.x % P), edges);
        part[kPartSweep * kPartStride + blockIdx.x] = edges;
        part[kPartDeg * kPartStride + blockIdx.x] = degsum;
        if (kDefer && removed) add_dev(ctr + kHyDead0 + 1, (int)removed);
    }
}

// ------------------------------------------ late support registration
// With opts.rounds = R >= 2 the first R - 1 rounds are AC-3 rounds with the
// edge_index cursor (Sections 4.1 and 8): no vertex joins a list.  Round 1 is
// ac6_sweep<kDefer>, which, like the plain first sweep, finds the vertices
// without successors removed already, so a vertex of peeling level l >= 2 is
// removed in round l - 1.  Round r >= 2 (ac6_round) takes the list of the vertices
// still live, each with its cursor target, and re-checks that target against
// the removals of rounds before r; a removed target makes the vertex scan on.
// If a round removes nothing the fixed point is reached: every later launch
// returns at once and the live set is the complement of the round bitmap.
// Otherwise round R (kJoin) does the same check and registers each surviving
// vertex in the list of the target it stops at, exactly as the first sweep
// does (a plain exchange: nothing is closed while it runs); from there the
// forest collapse and the propagation run unchanged.  Every removal of a
// round is certain (its successors were all removed before), so the
// propagation starts from a state that a plain AC-6 run also passes through.
//
// Round bitmaps: two, y[0] and y[1].  Round r reads y[r & 1], which holds
// every removal of the rounds before r, and builds y[(r + 1) & 1], which held
// the removals before r - 1: it adds y[r & 1] word by word (the removals of
// round r - 1) and its own removals bit by bit.  A round never reads the
// bitmap it writes, so a removal of round r is seen from round r + 1 on,
// whatever the order of the lanes: the rounds, the removals of each and the
// number of successor checks are those of the sequential rounds.
//
// The round list: the vertices the first round left live, one entry each
// (vertex, cursor target with the flag bits above), two arrays of hcap ints,
// updated in place: an entry is written only when its cursor moves (the
// cursor position goes to cur[v]) or its vertex is removed.  A round reads
// every entry's target, and the vertex only where the target was removed;
// removals are few after the first rounds, so rewriting the list without
// them would cost more than skipping them.  The removal counts of the rounds
// rotate over three control words.
//
// Removal filters: a target found live in round r - 1 is removed before
// round r iff round r - 1 removed it, so each round also sets its removals
// in a hashed filter (RoundFilter, three slots in rotation) and the next
// round, while those removals are few, checks the filter (staged in LDS)
// first and the round bitmap only on a hit.

// True (and the stop word set) if round r need not run: a round before it
// removed nothing.  Every workgroup decides from the same count, which no one
// changes while this kernel runs; only workgroup 0 writes the stop word (a
// store from each of thousands of workgroups to one word queues them all).
__device__ __forceinline__ bool deferred_done(int* ctr, int r) {
    if (ld_dev(ctr + kHyStop)) return true;
    if (ld_dev(ctr + kHyDead0 + (r - 1) % 3) == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st_dev(ctr + kHyStop, 1);
        return true;
    }
    return false;
}

constexpr int kRoundUnroll = 4;   // list entries per thread in flight

template <class View, bool kJoin>
__global__ __launch_bounds__(256) void ac6_round(View g, int r, const uint32_t* ycur,
                                                 uint32_t* ynext, int nwords, int* lst,
                                                 long long hcap, int* cur, RoundFilter flt,
                                                 int* head, int* ext, uint64_t* rec, int* jp,
                                                 uint32_t* jlist, uint32_t* q, int* ctr,
                                                 uint64_t* worker_edges, int P, int sched) {
    constexpr int U = kRoundUnroll;
    __shared__ uint64_t lds[Stage<View>::kWords];
    __shared__ uint32_t buf[kJoin ? U * 256 : 1];
    __shared__ uint32_t sflt[1 << (kRoundFilterMaxLog2 - 5)];   // round r - 1's filter
    __shared__ int s_base, s_nbuf;
    __shared__ uint64_t red[16];
    if (deferred_done(ctr, r)) return;
    Stage<View>::apply(g, lds);
    const int cnt = ld_dev(ctr + kHyCnt0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st_dev(ctr + kHyDead0 + (r + 1) % 3, 0);
        st_dev(ctr + kHyRounds, r);
    }
    const int stride = gridDim.x * blockDim.x;
    // Every live entry's target was found live against the removals before
    // round r - 1, so it is removed before round r iff round r - 1 removed
    // it: while those removals are few, their filter (L2-resident) answers
    // most checks and only its hits read the round bitmap.
    const bool use_flt =
        flt.f && ld_dev(ctr + kHyDead0 + (r - 1) % 3) <= (1 << flt.log2) / 8;
    if (use_flt) {   // staged in LDS: the checks then leave L2 alone
        const uint32_t* fs = flt.slot(r - 1);
        for (int i = threadIdx.x; i < flt.words(); i += blockDim.x) sflt[i] = fs[i];
        __syncthreads();
    }
    if constexpr (!kJoin) {
        // the removals of round r - 1 into the bitmap this round builds, and
        // the filter slot round r + 1 writes cleared
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) {
            const uint32_t b = ycur[i];
            if (b && (b & ~ynext[i])) atomicOr(ynext + i, b);
        }
        if (flt.f)
            for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < flt.words(); i += stride)
                flt.slot(r + 1)[i] = 0;
    } else {
        if (threadIdx.x == 0) s_nbuf = 0;
        __syncthreads();
    }
    int* lv = lst;
    int* lt = lst + hcap;
    uint64_t edges = 0, removed = 0, entries = 0;
    for (int base = blockIdx.x * blockDim.x * U; base < cnt; base += stride * U) {
        int v[U], p[U];
        uint32_t t[U];
        bool keep[U], gone[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = base + k * blockDim.x + threadIdx.x;
            t[k] = kGoneBit;
            if (i < cnt) t[k] = (uint32_t)__builtin_nontemporal_load(lt + i);
        }
        // the cursor targets' bits; a registering round needs every entry's
        // vertex, the others only the vertices whose target was removed
        bool moved[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int w = (int)(t[k] & kTargetMask);
            bool hit = true;
            if (use_flt) {
                const uint32_t h = flt.hash(w);
                hit = (sflt[h >> 5] >> (h & 31)) & 1u;
            }
            moved[k] = !(t[k] & kGoneBit) && hit && ((ycur[w >> 5] >> (w & 31)) & 1u);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = base + k * blockDim.x + threadIdx.x;
            v[k] = -1;
            if (!(t[k] & kGoneBit) && (kJoin || moved[k]))
                v[k] = __builtin_nontemporal_load(lv + i);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            keep[k] = gone[k] = false;
            if (t[k] & kGoneBit) continue;
            entries += 1;
            p[k] = -1;   // unchanged cursor (read only where needed)
            if (!moved[k]) {   // the cursor edge, checked again: its target is live
                edges += 1;
                keep[k] = kJoin;
                continue;
            }
            // the cursor target was removed before this round: scan on
            const int p0 = (t[k] & kFirstBit) ? g.begin(v[k]) : cur[v[k]];
            const int e1 = g.end(v[k]);
            const int ctx = g.vctx(v[k]);
            int pp = p0 + 1, x = 0;
            for (; pp < e1; ++pp) {
                x = g.target(v[k], pp, ctx);
                if (!((ycur[x >> 5] >> (x & 31)) & 1u)) break;
            }
            const int i = base + k * blockDim.x + threadIdx.x;
            if (pp < e1) {
                edges += (uint64_t)(pp - p0 + 1);
                t[k] = (uint32_t)x | (pp + 1 == e1 ? kLastBit : 0u);
                p[k] = pp;
                if constexpr (!kJoin) {
                    cur[v[k]] = pp;
                    lt[i] = (int)t[k];
                }
                keep[k] = true;
            } else {
                edges += (uint64_t)(e1 - p0);
                gone[k] = true;
                if constexpr (!kJoin) lt[i] = (int)(t[k] | kGoneBit);
            }
        }
        if constexpr (!kJoin) {
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (gone[k]) {
                    atomicOr(ynext + (v[k] >> 5), 1u << (v[k] & 31));
                    if (flt.f) flt.add(r, v[k]);
                    removed += 1;
                }
            }
        } else {
            // register the survivors (the joins' round trips overlap), list the
            // removed vertices and the tree members for the forest collapse
            // (or queue the removed ones as close items without it)
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (keep[k] && p[k] < 0)
                    p[k] = (t[k] & kFirstBit) ? g.begin(v[k]) : cur[v[k]];
            int old[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (keep[k]) {
                    if (sched & TRIM_SCHED_JITTER)
                        jitter_nap(((uint64_t)blockIdx.x << 32) ^ (uint32_t)v[k]);
                    const int w = (int)(t[k] & kTargetMask);
                    old[k] = xchg_dev(join_slot(head, ext, w, (t[k] & kLastBit) != 0u, v[k]), v[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                bool member = false;
                if (keep[k]) {
                    rec[v[k]] = pack_rec(old[k], p[k]);
                    member = (t[k] & kLastBit) != 0u;
                    if (jp) jp[v[k]] = member ? (int)(t[k] & kTargetMask) : v[k];
                } else if (gone[k] && jp) {
                    jp[v[k]] = ~v[k];
                }
                const bool put = gone[k] || (jp && member);
                const uint64_t mask = ballot(put);
                if (mask) {
                    int wbase = 0;
                    if (lane_id() == 0) wbase = atomicAdd(&s_nbuf, popc(mask));
                    wbase = __shfl(wbase, 0);
                    if (put)
                        buf[wbase + popc(mask & lanes_below())] =
                            jp ? ((uint32_t)v[k] | (gone[k] ? kRootBit : 0u))
                               : make_item(0, v[k]);
                }
            }
            // one reservation per step for what the block buffered
            __syncthreads();
            const int nb = s_nbuf;
            if (nb > 0) {
                if (threadIdx.x == 0) {
                    if (jp) {
                        s_base = add_dev(ctr + kJCnt0, nb);
                    } else {
                        add_dev(ctr + kPending, nb);
                        s_base = add_dev(ctr + kQTail, nb);
                    }
                }
                __syncthreads();
                uint32_t* dst = jp ? jlist : q;
                for (int j = threadIdx.x; j < nb; j += blockDim.x) dst[s_base + j] = buf[j];
                __syncthreads();
                if (threadIdx.x == 0) s_nbuf = 0;
            }
            __syncthreads();
        }
    }
    edges = block_sum(edges, red);
    entries = block_sum(entries, red);
    if constexpr (!kJoin) removed = block_sum(removed, red);
    if (threadIdx.x == 0) {
        if (edges) add_dev(worker_edges + (blockIdx.x % P), edges);
        if (entries) add_dev(reinterpret_cast<uint64_t*>(ctr + kHyWork), entries);
        if (!kJoin && removed) add_dev(ctr + kHyDead0 + r % 3, (int)removed);
    }
}

// The list heads before round R registers supports: kDead (closed) for every
// vertex removed so far -- the sinks, the preset vertices and the removals of
// the rounds -- and kEmpty for the others.
__global__ void ac6_heads(int n, int r, const uint32_t* y, int* head, int* ext, int* ctr) {
    if (deferred_done(ctr, r)) return;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int h = ((y[v >> 5] >> (v & 31)) & 1u) ? kDead : kEmpty;
        reinterpret_cast<int2*>(head)[v] = make_int2(h, h);
        if (ext)
            for (int j = 0; j < kMoreLists - 1; ++j) ext[(kMoreLists - 1) * (long long)v + j] = h;
    }
}

// Work items of the propagation:
//   CLOSE(x)       x found no live successor: close both of its lists;
//   CLOSE_LAST(x)  the same for a member x of some S_last(p): x is removed with
//                  p, and x's record links to the next member of S_last(p);
//   WALK(x)        x heads (the rest of) a closed S_more list: follow the links
//                  and hand each member out as a RESCAN item, up to kWalk
//                  members in a row.  The walk only loads links (one memory
//                  round trip per member), so a long list -- a hub's -- is not
//                  walked at the pace of its members' rescans;
//   RESCAN(x)      x was in a closed S_more list: resume its DoPost after its
//                  old support (edge_index, Section 8).
// RESCAN items go to the wave-local ring: the other lanes of the walking
// wave rescan while the walker goes on, and the shared queue never holds
// them (it has room for three items per vertex; hand-backs are only bounded
// by the number of joins).  A full local ring stops the walk until it drains.
enum : uint32_t { kClose = 0, kCloseLast = 1, kWalkMore = 2, kRescan = 3 };
constexpr int kHops = 256;   // S_last chain steps one item may take in a row
constexpr int kWalk = 32;    // S_more members one WALK item hands out in a row

template <class View>
__global__ __launch_bounds__(256) void ac6_propagate(View g, int* head, int* ext, uint64_t* rec,
                                                     uint32_t* q, int* ctr,
                                                     uint64_t* worker_edges, uint64_t* part,
                                                     int sched, int budget) {
    __shared__ uint64_t lds[Stage<View>::kWords];
    __shared__ uint32_t rings[256 / kWave][kLocalQ];
    __shared__ int ring_tail[256 / kWave];
    __shared__ uint32_t local_rings[256 / kWave][kLocalP];
    __shared__ int local_tail[256 / kWave];
    __shared__ uint64_t red[16];
    if (ld_dev(ctr + kHyStop)) {   // the rounds reached the fixed point: nothing to do
        if (threadIdx.x == 0)
            for (int slot : {kPartCloses, kPartJoins, kPartVisited, kPartQhw})
                part[slot * kPartStride + blockIdx.x] = 0;
        return;
    }
    Stage<View>::apply(g, lds);
    WaveQueue wq;
    const int wv = threadIdx.x / kWave;
    wq.init(rings[wv], &ring_tail[wv], q, ctr + kQHead, ctr + kQTail, ctr + kPending,
            ctr + kStall, budget, ShareEvery<View>::value, local_rings[wv], &local_tail[wv]);
    uint32_t item = kNone;
    uint64_t edges = 0, closes = 0, joins = 0, visited = 0;
    while (wq.acquire(item)) {
        uint32_t keep = kNone;
        // A walk member that finds no live successor is closed in the same
        // iteration (its next member goes to the ring instead), so a peeling
        // step through a supporter list costs one queue round, not two.
        bool close_now = false;
        int cx = 0;
        bool member = false;
        if (item != kNone) {
            const int x = item_vertex(item);
            const uint32_t kind = item_kind(item);
            int rx = -1, cont = -1;   // a member rescanned by this lane now; the rest of its list
            if (kind == kWalkMore) {
                // Each link is read before its member is handed out (a rescan
                // that re-joins rewrites the member's record).  The last
                // member of a burst, and any member the full local ring does
                // not take, is rescanned by the walker itself, so every
                // iteration makes progress.
                int y = x;
                for (int h = 0;; ++h) {
                    const int ny = ld_dev(rec_link(rec, y));
                    visited += 1;
                    if (h + 1 < kWalk && wq.push_local(make_item(kRescan, y))) {
                        if (ny < 0) break;
                        y = ny;
                        continue;
                    }
                    rx = y;
                    cont = ny;
                    break;
                }
            } else if (kind == kRescan) {
                rx = x;
            } else {
                close_now = true;
                cx = x;
                member = kind == kCloseLast;
            }
            if (rx >= 0) {
                // rx is in no list until it joins again: its record is stable
                const uint64_t r = ld_dev(rec + rx);
                if (sched & TRIM_SCHED_JITTER) jitter_nap(rx);
                if (resume(g, rx, rec_cursor(r) + 1, head, rec, edges, sched, ext)) {
                    joins += 1;
                    if (cont >= 0) keep = make_item(kWalkMore, cont);
                } else {
                    if (cont >= 0) wq.push1(make_item(kWalkMore, cont));
                    close_now = true;
                    cx = rx;
                }
            }
        }
        if (close_now) {
            // Close cx, then follow S_last: its members have no successor left,
            // so each is removed at once.  One step = one exchange of both list
            // heads plus, for an S_last member, the load of its list link --
            // both in flight together, one round trip.  The next step's memory
            // operations are issued before this step's pushes, so the LDS queue
            // work overlaps the round trip.  Only the link half of a record is
            // loaded: a 32-bit load, so no register of an in-flight load is
            // reused by the pushes below.
            int link = member ? ld_dev(rec_link(rec, cx)) : -1;
            ClosedLists cl = close_lists(head, ext, cx);   // S_more(cx), S_last(cx)
            int fill = 0;   // ring fill read after the previous step's pushes
            for (int hop = 0;; ++hop) {
                closes += 1;
                // a dying vertex never joins a list again, so its record is stable
                const int sib = member ? link : -1;
                const ClosedLists cur = cl;
                const int b = cur.last;
                // depth first: into S_last(c) if it has members, else on to the
                // next member of the list c was in
                const int next = b >= 0 ? b : sib;
                visited += (b >= 0) + (sib >= 0);
                const bool go = next >= 0 && hop + 1 < kHops && fill <= kLocalQ - 256;
                if (go) {
                    if (sched & TRIM_SCHED_JITTER) jitter_nap(((uint64_t)next << 8) ^ hop);
                    link = ld_dev(rec_link(rec, next));
                    cl = close_lists(head, ext, next);
                }
#pragma unroll
                for (int j = 0; j < kMoreLists; ++j)
                    if (cur.more[j] >= 0) wq.push1(make_item(kWalkMore, cur.more[j]));
                if (b >= 0 && sib >= 0) wq.push1(make_item(kCloseLast, sib));
                fill = wq.fill();
                if (!go) {
                    if (next >= 0) keep = make_item(kCloseLast, next);
                    break;
                }
                member = true;
            }
        }
        item = keep;
        wq.rebalance();
    }
    edges = block_sum(edges, red);
    closes = block_sum(closes, red);
    joins = block_sum(joins, red);
    visited = block_sum(visited, red);
    const int qhw = block_max(wq.hw, reinterpret_cast<int*>(red));
    if (threadIdx.x == 0) {
        if (edges) add_dev(worker_edges + blockIdx.x, edges);
        part[kPartCloses * kPartStride + blockIdx.x] = closes;
        part[kPartJoins * kPartStride + blockIdx.x] = joins;
        part[kPartVisited * kPartStride + blockIdx.x] = visited;
        part[kPartQhw * kPartStride + blockIdx.x] = (uint64_t)qhw;
    }
}

// Level-synchronous propagation: the bulk of the work after the first sweep
// (and the forest collapse) runs in phases, the frontier form of Table
// trim-2.  A phase processes every item of its list -- CLOSE(x): exchange
// both of x's list heads with kDead and hand back both lists; RESCAN(x):
// resume x's DoPost after its old support, and close x if it finds none;
// WALK(x): hand back the S_more list headed by x -- and writes the items it
// creates to the next phase's list: a CLOSE for every S_last member (it has
// no successor left) and a RESCAN for every S_more member.  The lists are
// walked in lockstep, one link per lane per step; created items are staged
// per wavefront in LDS and reserved in the next list with one fetch-add per
// flush.  A grid barrier ends each phase.  Nothing here touches the shared
// ticket queue, whose few counters every wavefront would otherwise contend
// for.  Once a phase's list is shorter than kTailItems (a deep, narrow
// remainder, such as a chain), its items go to the shared queue and the
// asynchronous kernel finishes: it follows a chain at one memory round trip
// per removal, where a phase costs a barrier.  Launched with at most two
// workgroups per CU, all resident at once.
constexpr int kTailItems = 256;
constexpr int kStage = 256;   // items staged per wavefront before one reservation

template <class View>
__global__ __launch_bounds__(256) void ac6_levels(View g, int* head, int* ext, uint64_t* rec, uint32_t* q,
                                                  uint32_t* l0, uint32_t* l1, int* ctr,
                                                  uint64_t* worker_edges, int P, uint64_t* part,
                                                  int sched, int budget) {
    __shared__ uint64_t lds[Stage<View>::kWords];
    __shared__ uint32_t stage[256 / kWave][kStage];
    __shared__ int stage_n[256 / kWave];
    __shared__ uint64_t red[16];
    if (ld_dev(ctr + kHyStop)) {   // the rounds reached the fixed point: nothing to do
        if (threadIdx.x == 0)
            for (int slot : {kPartLvCloses, kPartLvJoins, kPartLvVisited})
                part[slot * kPartStride + blockIdx.x] = 0;
        return;
    }
    Stage<View>::apply(g, lds);
    const int wv = threadIdx.x / kWave;
    if (lane_id() == 0) stage_n[wv] = 0;
    __builtin_amdgcn_wave_barrier();
    uint64_t edges = 0, closes = 0, joins = 0, visited = 0;
    const int stride = gridDim.x * blockDim.x;
    int* out_cnt = nullptr;
    uint32_t* out = nullptr;
    // move this wavefront's staged items to the next list (wave-uniform)
    auto flush = [&]() {
        const int k = stage_n[wv];
        if (k == 0) return;
        int base = 0;
        if (lane_id() == 0) base = add_dev(out_cnt, k);
        base = __shfl(base, 0);
        for (int i = lane_id(); i < k; i += kWave) st_dev((int*)out + base + i, (int)stage[wv][i]);
        __builtin_amdgcn_wave_barrier();
        if (lane_id() == 0) stage_n[wv] = 0;
        __builtin_amdgcn_wave_barrier();
    };
    // stage this lane's item, if any (wave-uniform)
    auto emit = [&](uint32_t e) {
        const uint64_t mk = ballot(e != kNone);
        const int k = popc(mk);
        if (k == 0) return;
        if (stage_n[wv] + k > kStage) flush();
        const int base = stage_n[wv];
        if (e != kNone) stage[wv][base + popc(mk & lanes_below())] = e;
        __builtin_amdgcn_wave_barrier();
        if (lane_id() == 0) stage_n[wv] = base + k;
        __builtin_amdgcn_wave_barrier();
    };
    const int n0 = ld_dev(ctr + kQTail);   // the first phase's items, in the shared queue
    for (int ph = 0;; ++ph) {
        const uint32_t* in = ph == 0 ? q : ((ph & 1) ? l0 : l1);
        const int cnt = ph == 0 ? n0 : ld_dev(ctr + kLvCnt0 + ph % 3);
        if (cnt < kTailItems) {
            // the rest goes to the asynchronous kernel, through the shared queue
            if (ph > 0) {
                for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride)
                    st_dev((int*)q + i, ld_dev((const int*)in + i));
                if (blockIdx.x == 0 && threadIdx.x == 0) {
                    st_dev(ctr + kQHead, 0);
                    st_dev(ctr + kQTail, cnt);
                    st_dev(ctr + kPending, cnt);
                }
            }
            break;
        }
        out = (ph & 1) ? l1 : l0;
        out_cnt = ctr + kLvCnt0 + (ph + 1) % 3;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st_dev(ctr + kLvCnt0 + (ph + 2) % 3, 0);
            add_dev(ctr + kLvPhases, 1);
        }
        for (int base = blockIdx.x * blockDim.x; base < cnt; base += stride) {
            const int i = base + threadIdx.x;
            uint32_t it = kNone;
            if (i < cnt) {
                it = (uint32_t)ld_dev((const int*)in + i);
                if (ph == 0) st_dev((int*)q + i, (int)kNone);   // the slot is free again
            }
            // the chains this lane walks: S_last (CLOSE items) and the S_more
            // lists (RESCAN items), all advanced together
            int walk_last = -1, cx = -1;
            int walk_more[kMoreLists];
#pragma unroll
            for (int j = 0; j < kMoreLists; ++j) walk_more[j] = -1;
            if (it != kNone) {
                const int x = item_vertex(it);
                const uint32_t kind = item_kind(it);
                if (kind == kWalkMore) {
                    walk_more[0] = x;
                } else if (kind == kRescan) {
                    // x is in no list until it joins again: its record is stable
                    const uint64_t r = ld_dev(rec + x);
                    if (sched & TRIM_SCHED_JITTER) jitter_nap(x);
                    if (resume(g, x, rec_cursor(r) + 1, head, rec, edges, sched, ext))
                        joins += 1;
                    else
                        cx = x;
                } else {
                    cx = x;   // a close (the first phase's items are closes or walks)
                }
            }
            if (cx >= 0) {
                if (sched & TRIM_SCHED_JITTER) jitter_nap((uint64_t)cx << 8);
                const ClosedLists cl = close_lists(head, ext, cx);
                closes += 1;
#pragma unroll
                for (int j = 0; j < kMoreLists; ++j) walk_more[j] = cl.more[j];
                walk_last = cl.last;
            }
            // a member's link is read before its item exists: its own processing,
            // in the next phase, is the only thing that can change its record
            auto active = [&]() {
                bool a = walk_last >= 0;
#pragma unroll
                for (int j = 0; j < kMoreLists; ++j) a = a || walk_more[j] >= 0;
                return a;
            };
            while (ballot(active())) {
                int nl = -1, nm[kMoreLists];
                if (walk_last >= 0) nl = ld_dev(rec_link(rec, walk_last));
#pragma unroll
                for (int j = 0; j < kMoreLists; ++j)
                    nm[j] = walk_more[j] >= 0 ? ld_dev(rec_link(rec, walk_more[j])) : -1;
                visited += walk_last >= 0;
                emit(walk_last >= 0 ? make_item(kClose, walk_last) : kNone);
                walk_last = nl;
#pragma unroll
                for (int j = 0; j < kMoreLists; ++j) {
                    visited += walk_more[j] >= 0;
                    emit(walk_more[j] >= 0 ? make_item(kRescan, walk_more[j]) : kNone);
                    walk_more[j] = nm[j];
                }
            }
        }
        flush();
        if (!grid_barrier(ctr + kBarCount, ctr + kBarGen, ctr + kStall, budget)) break;
    }
    edges = block_sum(edges, red);
    closes = block_sum(closes, red);
    joins = block_sum(joins, red);
    visited = block_sum(visited, red);
    if (threadIdx.x == 0) {
        if (edges) add_dev(worker_edges + (blockIdx.x % P), edges);
        part[kPartLvCloses * kPartStride + blockIdx.x] = closes;
        part[kPartLvJoins * kPartStride + blockIdx.x] = joins;
        part[kPartLvVisited * kPartStride + blockIdx.x] = visited;
    }
}

// The forest collapse's removal (the jump kernel is in forest_jump.h): both
// heads of v exchanged with kDead, its S_more lists handed to the propagation
// as walk items.
struct OneSidedKill {
    int* head;
    int* ext;
    __device__ __forceinline__ void operator()(int v, uint32_t (&item)[kJumpItems]) const {
        const ClosedLists cl = close_lists(head, ext, v);
#pragma unroll
        for (int j = 0; j < kMoreLists; ++j)
            if (cl.more[j] >= 0) item[j] = make_item(kWalkMore, cl.more[j]);
    }
};

struct Ac6Live {
    const int* head;
    __device__ __forceinline__ bool operator()(int v) const { return head[2 * v] != kDead; }
};

// The live bitmap with late support registration: the complement of the
// round bitmap when the rounds reached the fixed point (no support was
// registered), else from the list heads as after a plain run.
__global__ void ac6_pack_deferred(const int* head, const uint32_t* y, int n, uint32_t* bitmap,
                                  uint64_t* part, const int* ctr, uint32_t* q, long long qwords) {
    __shared__ uint64_t red[16];
    clear_queue_if_stalled(ctr, q, qwords);
    const int nwords = (n + 31) >> 5;
    uint64_t live_cnt = 0;
    if (ld_dev(ctr + kHyStop)) {
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
             i += gridDim.x * blockDim.x) {
            uint32_t wd = ~y[i];
            if (i == nwords - 1 && (n & 31)) wd &= (1u << (n & 31)) - 1u;
            bitmap[i] = wd;
            live_cnt += (uint64_t)__popc(wd);
        }
    } else {
        const int waves = (gridDim.x * blockDim.x) / kWave;
        const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
        for (int base = wid * kWave; base < n; base += waves * kWave) {
            const int v = base + lane_id();
            const uint64_t b = ballot(v < n && head[2 * v] != kDead);
            if (lane_id() == 0) {
                const int w = base >> 5;
                bitmap[w] = (uint32_t)b;
                if (w + 1 < nwords) bitmap[w + 1] = (uint32_t)(b >> 32);
                live_cnt += (uint64_t)popc(b);
            }
        }
    }
    live_cnt = block_sum(live_cnt, red);
    if (threadIdx.x == 0) part[kPartLive * kPartStride + blockIdx.x] = live_cnt;
}

// Per-graph bitmaps: word wi of the packed output belongs to graph g with
// bitmap_base[g] <= wi < bitmap_base[g+1] and covers local vertices
// 32 * (wi - bitmap_base[g]) .. + 31 (bits past the graph's n are zero).
__global__ void ac6_pack_batch(const int* head, const int64_t* vbase, const int64_t* bitmap_base,
                               int G, uint32_t* bitmaps, uint64_t* part, const int* ctr,
                               uint32_t* q, long long qwords) {
    __shared__ uint64_t red[16];
    clear_queue_if_stalled(ctr, q, qwords);
    const int64_t total_words = bitmap_base[G];
    uint64_t live_cnt = 0;
    for (int64_t wi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; wi < total_words;
         wi += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = G - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (bitmap_base[mid] <= wi) lo = mid; else hi = mid - 1;
        }
        const int64_t v0 = vbase[lo];
        const int64_t ng = vbase[lo + 1] - v0;
        const int64_t l0 = (wi - bitmap_base[lo]) * 32;
        uint32_t word = 0;
        for (int j = 0; j < 32; ++j) {
            const int64_t l = l0 + j;
            if (l < ng && head[2 * (v0 + l)] != kDead) word |= 1u << j;
        }
        bitmaps[wi] = word;
        live_cnt += (uint64_t)__popc(word);
    }
    live_cnt = block_sum(live_cnt, red);
    if (threadIdx.x == 0) part[kPartLive * kPartStride + blockIdx.x] = live_cnt;
}

// base[v] = first vertex of v's graph (one block per graph).
__global__ void batch_bases(const int64_t* vbase, int G, int* base) {
    for (int gi = blockIdx.x; gi < G; gi += gridDim.x) {
        const int v0 = (int)vbase[gi], v1 = (int)vbase[gi + 1];
        for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) base[v] = v0;
    }
}

// Traversed edges of each graph, read off the final state: a removed vertex
// checked all its successors, a live one every position up to its support
// (its cursor).  AC-6's total does not depend on the schedule, so this equals
// the number of checks the run made.
__global__ void batch_graph_edges(const int* head, const uint64_t* rec, const int* row_off,
                                  const int64_t* vbase, int G, uint64_t* graph_edges) {
    __shared__ uint64_t red[16];
    for (int gi = blockIdx.x; gi < G; gi += gridDim.x) {
        const int v0 = (int)vbase[gi], v1 = (int)vbase[gi + 1];
        uint64_t s = 0;
        for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
            const int b = row_off[v], e = row_off[v + 1];
            if (head[2 * v] == kDead) s += (uint64_t)(e - b);
            else s += (uint64_t)(rec_cursor(rec[v]) - b + 1);
        }
        s = block_sum(s, red);
        if (threadIdx.x == 0) graph_edges[gi] = s;
        __syncthreads();
    }
}

inline int grid_for(long long n, int block, int max_blocks = 1 << 20) {
    long long b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

// Which views take ac6_init_bits: explicit graphs whose offsets are 16-byte
// aligned (the caller's pointer; torch allocations are).
template <class View>
struct InitBits {
    static bool ok(const View&) { return false; }
    static const int* row_off(const View&) { return nullptr; }
};
template <>
struct InitBits<ExplicitView> {
    static bool ok(const ExplicitView& g) { return ((uintptr_t)g.row_off & 15) == 0; }
    static const int* row_off(const ExplicitView& g) { return g.row_off; }
};

// Words from the first round bitmap to the second (both in w.c, which holds
// n + n / 8 + 64 ints): room for ceil(n / 32) words plus the one past the end
// that ac6_init may write, aligned to a cache line.
inline long long round_bitmap_offset(long long n) { return ((n + 31) / 32 + 2 + 31) / 32 * 32; }
// Workgroups of a round launch: about one per 1,024 list entries (a list
// holds at most n), at most four per CU
// (more workgroups measured slower: every round launch after the fixed point
// still starts them all).
inline int round_blocks(long long n, int cus) {
    long long b = (n + 256 * kRoundUnroll - 1) / (256 * kRoundUnroll);
    if (b < 1) b = 1;
    if (b > 4LL * cus) b = 4LL * cus;
    return (int)b;
}

template <class View>
hipError_t ac6_run(View g, int n, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                   uint64_t* worker_edges, trim_stats_t* stats, const int64_t* vbase = nullptr,
                   const int64_t* bitmap_base = nullptr, int G = 0,
                   const uint32_t* preset = nullptr) {
    const int P = lc.workers;
    const int B = lc.block;
    int sweep_blocks = 0, pack_blocks = 0, level_blocks = 0;
    // split S_more lists for graphs up to kSplitMaxN vertices (their extra
    // heads exist only then)
    int* ext = (w.ext && n <= kSplitMaxN) ? w.ext : nullptr;
    // late support registration: R rounds, two round bitmaps in w.c (y[1] is
    // the sinks bitmap the first round reads), the round list in w.hl
    const int R = (!bitmap_base && w.hl && w.hcap >= n) ? lc.rounds : 0;
    const bool defer = R >= 2;
    uint32_t* y[2];
    y[1] = reinterpret_cast<uint32_t*>(w.c);
    y[0] = y[1] + round_bitmap_offset(n);
    const int nwords = (n + 31) / 32;
    // the round filters follow the round list in w.hl: 2^flog bits each, about
    // n / 8 bits (at least 32, at most kRoundFilterMaxLog2)
    RoundFilter flt;
    if (defer) {
        flt.f = reinterpret_cast<uint32_t*>(w.hl + 2 * w.hcap);
        int flog = 5;
        while (flog < kRoundFilterMaxLog2 && (1LL << (flog + 3)) < (long long)n) ++flog;
        flt.log2 = flog;
    }
    {
        Timed t(lc, "ac6_init");
        if (defer && InitBits<View>::ok(g))
            hipLaunchKernelGGL(ac6_init_bits, dim3(grid_for((n + 3) / 4, 256, 16384)), dim3(256),
                               0, lc.stream, InitBits<View>::row_off(g), n, y[1], y[0], w.ctr,
                               worker_edges, P, stats, flt);
        else
            hipLaunchKernelGGL(ac6_init<View>, dim3(grid_for(n, 256, 16384)), dim3(256), 0,
                               lc.stream, g, n, defer ? nullptr : w.a, ext, y[1],
                               defer ? y[0] : nullptr, preset, w.ctr, worker_edges, P, stats,
                               flt);
    }
    if (n > 0) {
        const int chunk = sweep_chunk(lc, n, B);
        sweep_blocks = grid_for(n, chunk, lc.cus * 8);
        if (!defer) {
            Timed t(lc, "ac6_sweep");
            hipLaunchKernelGGL((ac6_sweep<View, false>), dim3(sweep_blocks), dim3(B), 0, lc.stream,
                               g, n, chunk, w.a, ext, y[1], preset, w.b, w.q, w.ctr, worker_edges,
                               P, w.part, lc.schedule, lc.forest ? w.jp : nullptr,
                               lc.forest ? w.e : nullptr, nullptr, nullptr, 0LL, nullptr, flt);
        } else {
            // the round list in w.hl, the moved cursors in w.d
            {
                Timed t(lc, "ac6_sweep");
                hipLaunchKernelGGL((ac6_sweep<View, true>), dim3(sweep_blocks), dim3(B), 0,
                                   lc.stream, g, n, chunk, nullptr, nullptr, y[1], preset, w.b,
                                   w.q, w.ctr, worker_edges, P, w.part, lc.schedule, nullptr,
                                   nullptr, y[0], w.hl, w.hcap, w.d, flt);
            }
            const int rb = round_blocks(n, lc.cus);
            if (R > 2) {
                Timed t(lc, "ac6_rounds");
                for (int r = 2; r < R; ++r)
                    hipLaunchKernelGGL((ac6_round<View, false>), dim3(rb), dim3(256), 0,
                                       lc.stream, g, r, y[r & 1], y[(r + 1) & 1], nwords, w.hl,
                                       w.hcap, w.d, flt, nullptr, nullptr, nullptr, nullptr,
                                       nullptr, nullptr, w.ctr, worker_edges, P, lc.schedule);
            }
            {
                Timed t(lc, "ac6_register");
                hipLaunchKernelGGL(ac6_heads, dim3(grid_for(n, 256, 16384)), dim3(256), 0,
                                   lc.stream, n, R, y[R & 1], w.a, ext, w.ctr);
                hipLaunchKernelGGL((ac6_round<View, true>), dim3(rb), dim3(256), 0, lc.stream, g,
                                   R, y[R & 1], nullptr, nwords, w.hl, w.hcap, w.d, flt, w.a, ext,
                                   w.b, lc.forest ? w.jp : nullptr, lc.forest ? w.e : nullptr,
                                   w.q, w.ctr, worker_edges, P, lc.schedule);
            }
        }
        if (lc.forest) {
            Timed t(lc, "ac6_jump");
            hipLaunchKernelGGL(ac6_jump<OneSidedKill>, dim3(phase_blocks(n, lc.cus)), dim3(256), 0,
                               lc.stream, OneSidedKill{w.a, ext}, w.jp, w.e, w.e + n, w.q, w.ctr,
                               jump_rounds(n), lc.budget);
        }
        level_blocks = phase_blocks(n, lc.cus);
        {
            Timed t(lc, "ac6_levels");
            hipLaunchKernelGGL(ac6_levels<View>, dim3(level_blocks), dim3(256), 0, lc.stream, g,
                               w.a, ext, w.b, w.q, w.e, w.e + n, w.ctr, worker_edges, P, w.part,
                               lc.schedule, lc.budget);
        }
        {
            Timed t(lc, "ac6_propagate");
            hipLaunchKernelGGL(ac6_propagate<View>, dim3(P), dim3(256), 0, lc.stream, g, w.a,
                               ext, w.b, w.q, w.ctr, worker_edges, w.part, lc.schedule, lc.budget);
        }
        if (!bitmap_base) {
            Timed t(lc, "ac6_pack");
            pack_blocks = grid_for(n, 256, lc.cus * 4);
            if (defer)
                hipLaunchKernelGGL(ac6_pack_deferred, dim3(pack_blocks), dim3(256), 0, lc.stream,
                                   w.a, y[0], n, bitmap, w.part, w.ctr, w.q, w.qwords);
            else
                hipLaunchKernelGGL(pack_bitmap<Ac6Live>, dim3(pack_blocks), dim3(256), 0,
                                   lc.stream, Ac6Live{w.a}, n, bitmap, w.part, w.ctr, w.q,
                                   w.qwords);
        }
    }
    if (bitmap_base && n > 0) {
        Timed t(lc, "ac6_pack_batch");
        pack_blocks = grid_for(n / 32 + G, 256, lc.cus * 4);
        hipLaunchKernelGGL(ac6_pack_batch, dim3(pack_blocks), dim3(256), 0, lc.stream, w.a,
                           vbase, bitmap_base, G, bitmap, w.part, w.ctr, w.q, w.qwords);
    }
    if (stats) {
        Timed t(lc, "finalize");
        hipLaunchKernelGGL(finalize_stats, dim3(1), dim3(1024), 0, lc.stream, n, P, sweep_blocks,
                           n > 0 ? P : 0, pack_blocks, n > 0 ? P : 0, worker_edges, w.part,
                           w.ctr, stats, 0, 0, level_blocks);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t ac6_csr(const trim_csr_t& g, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                   uint64_t* worker_edges, trim_stats_t* stats, const uint32_t* preset) {
    ExplicitView v{g.row_off, g.col};
    return ac6_run(v, g.n, w, lc, bitmap, worker_edges, stats, nullptr, nullptr, 0, preset);
}

hipError_t ac6_implicit(const trim_implicit_t& g, const Work& w, const LaunchCfg& lc,
                        uint32_t* bitmap, uint64_t* worker_edges, trim_stats_t* stats) {
    const int n = 1 << g.log2n;
    ImplicitView v{g.seed, g.zero_thr, g.deg_table, (uint32_t)(n - 1)};
    return ac6_run(v, n, w, lc, bitmap, worker_edges, stats);
}

hipError_t ac6_batch(int G, const int64_t* vbase, const int32_t* row_off, const int32_t* col,
                     int64_t total_n, const int64_t* bitmap_base, const Work& w,
                     const LaunchCfg& lc, uint32_t* bitmaps, uint64_t* graph_edges,
                     trim_stats_t* stats) {
    const int gb = G < 16384 ? G : 16384;
    {
        Timed t(lc, "batch_bases");
        hipLaunchKernelGGL(batch_bases, dim3(gb), dim3(256), 0, lc.stream, vbase, G, w.d);
    }
    BatchView v{row_off, col, w.d};
    hipError_t e = ac6_run(v, (int)total_n, w, lc, bitmaps, w.wedges, stats, vbase, bitmap_base, G);
    if (e != hipSuccess) return e;
    Timed t(lc, "batch_graph_edges");
    hipLaunchKernelGGL(batch_graph_edges, dim3(gb), dim3(256), 0, lc.stream, w.a, w.b, row_off,
                       vbase, G, graph_edges);
    return hipGetLastError();
}

int ac6_max_workers_per_cu(int) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ac6_propagate<ExplicitView>, 256, 0) !=
        hipSuccess)
        return 1;
    int nb2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, ac6_propagate<ImplicitView>, 256, 0) ==
            hipSuccess &&
        nb2 < nb)
        nb = nb2;
    return nb < 1 ? 1 : nb;
}

}  // namespace trim
