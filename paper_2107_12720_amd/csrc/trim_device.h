// trim_device.h -- device-side building blocks shared by the trimming kernels.
//
// Memory-ordering protocol (gfx950, 8 XCDs with separate L2 caches).
// Agent-scope release/acquire orderings compile to whole-L2 write-back and
// invalidate instructions, far too costly per support registration.  The
// kernels instead use:
//  * device-coherent stores and loads (relaxed atomics at agent scope, which
//    bypass the non-coherent part of the cache hierarchy) for the few words
//    that one lane publishes to another: the (next, cursor) record of a
//    registered vertex and queue slots;
//  * `complete_mem()` -- an s_waitcnt vmcnt(0) with a compiler memory
//    barrier -- between such a store and the atomic that makes it reachable
//    (the CAS on a support list head, the queue tail bump), so the store has
//    been acknowledged at device scope before anyone can find it;
//  * device-scope atomic RMWs (CAS, exchange, add), which are coherent across
//    XCDs, for every contended word.
// Status reads while scanning successors may be stale: a stale read can only
// show an older, not-yet-removed value, and the CAS that follows fails and
// reloads.  DEAD is terminal, so it is never seen too early.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "trim_internal.h"

namespace trim {

constexpr int kEmpty = -1;   // support list head: no supporters yet
constexpr int kDead = -2;    // support list head: vertex removed, list closed
constexpr int kWave = 64;

__device__ __forceinline__ int ld_cached(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int ld_dev(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_dev(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_dev(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int xchg_dev(int* p, int v) {
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// On failure `expected` receives the current value.
// Exchange of an aligned pair of ints as one 8-byte atomic; returns the old
// pair (x = p[0], y = p[1]).
__device__ __forceinline__ int2 xchg2_dev(int* p, int v0, int v1) {
    const uint64_t v = ((uint64_t)(uint32_t)v1 << 32) | (uint32_t)v0;
    const uint64_t old = __hip_atomic_exchange(reinterpret_cast<uint64_t*>(p), v,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_int2((int)(uint32_t)old, (int)(uint32_t)(old >> 32));
}
__device__ __forceinline__ bool cas_dev(int* p, int& expected, int desired) {
    return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int add_dev(int* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned add_dev(unsigned* p, unsigned v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t add_dev(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The same operations at a chosen memory scope (a __HIP_MEMORY_SCOPE_* value):
// data that only one workgroup touches needs workgroup scope only, which the
// workgroup's own L2 serves.
template <int S>
__device__ __forceinline__ int ld_s(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ uint64_t ld_s(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ void st_s(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ int xchg_s(int* p, int v) {
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ int2 xchg2_s(int* p, int v0, int v1) {
    const uint64_t v = ((uint64_t)(uint32_t)v1 << 32) | (uint32_t)v0;
    const uint64_t old =
        __hip_atomic_exchange(reinterpret_cast<uint64_t*>(p), v, __ATOMIC_RELAXED, S);
    return make_int2((int)(uint32_t)old, (int)(uint32_t)(old >> 32));
}
template <int S>
__device__ __forceinline__ bool cas_s(int* p, int& expected, int desired) {
    return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, S);
}

// Wait until every vector memory operation this wave issued has completed.
__device__ __forceinline__ void complete_mem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc(uint64_t x) { return __popcll(x); }

__device__ __forceinline__ uint64_t wave_sum(uint64_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        unsigned lo = __shfl_xor((unsigned)x, off);
        unsigned hi = __shfl_xor((unsigned)(x >> 32), off);
        x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

// Record written by a vertex when it joins a support list: the previous list
// head (next supporter) in the low word, its cursor in the high word.
__device__ __forceinline__ uint64_t pack_rec(int next, int cursor) {
    return ((uint64_t)(uint32_t)cursor << 32) | (uint32_t)next;
}
__device__ __forceinline__ int rec_next(uint64_t r) { return (int)(uint32_t)r; }
__device__ __forceinline__ int rec_cursor(uint64_t r) { return (int)(uint32_t)(r >> 32); }
// Schedule perturbation (TRIM_SCHED_JITTER): a wavefront pauses for 0..7
// short naps, chosen by a hash of `salt`, inside a race window.
__device__ __forceinline__ void jitter_nap(uint64_t salt) {
    uint64_t z = salt * 0x9E3779B97F4A7C15ull;
    z ^= z >> 29;
    const int naps = (int)((z * 0xBF58476D1CE4E5B9ull) >> 61);
    for (int i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(2);
}

// The link half of rec[v] (the low word on this little-endian target).
__device__ __forceinline__ const int* rec_link(const uint64_t* rec, int v) {
    return reinterpret_cast<const int*>(rec + v);
}

// Wave-aggregated append of the lanes with `pred` set: one atomic per wave.
// Returns the slot of this lane (or -1).  Does not wait for completion.
__device__ __forceinline__ int wave_append_slot(bool pred, int* tail, int* pending) {
    uint64_t mask = ballot(pred);
    if (mask == 0) return -1;
    int leader = __ffsll((long long)mask) - 1;
    int cnt = popc(mask);
    int base = 0;
    if (lane_id() == leader) {
        if (pending) add_dev(pending, cnt);
        base = add_dev(tail, cnt);
    }
    base = __shfl(base, leader);
    return pred ? base + popc(mask & lanes_below()) : -1;
}

// ------------------------------------------------------------ work queues
// Items are 32-bit words: a 2-bit kind above a 30-bit vertex id.  kNone marks
// an empty lane and an empty global queue slot.
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kIdMask = 0x3FFFFFFFu;
__device__ __forceinline__ uint32_t make_item(uint32_t kind, int v) {
    return (kind << 30) | (uint32_t)v;
}
__device__ __forceinline__ uint32_t item_kind(uint32_t it) { return it >> 30; }
__device__ __forceinline__ int item_vertex(uint32_t it) { return (int)(it & kIdMask); }

constexpr int kLocalQ = 1024;             // LDS ring entries per wavefront
constexpr int kLocalP = 256;              // entries of the wave-local ring (never shared)
constexpr int kSpillAbove = kLocalQ / 2;  // ring fill that triggers a bulk hand-off
constexpr int kPollEvery = 64;            // busy iterations between shared-queue polls
constexpr int kMaxNaps = 4;               // idle back-off cap, in s_sleep(127) naps

// Work distribution of the persistent kernels (the paper's private waiting
// sets Q_p, Sections 5.2 / 6.2).  Each wavefront owns an LDS ring; items reach
// the shared queue only when a ring overflows or when some lane elsewhere is
// waiting for work.  A wavefront with nothing to do takes 64 tickets (one per
// lane) with a single fetch-add on qhead; ticket t is filled by whoever
// reserves slot t through qtail, so claims never retry.  `pending` counts
// shared-queue items plus wavefronts that hold private work: it reaches zero
// only when no work is left anywhere, and then waiting lanes give up.
// Watchdog: a wavefront that has looped `budget` times gives up and raises
// the stall word; every other wavefront sees it at its next idle poll (or
// within 256 busy iterations) and exits too, so the kernel always drains.
// Free slots hold kNone; a consumer resets the slot it took, so the buffer
// is clean for the next call without a fill pass.  Outstanding tickets are at
// most 64 per wavefront, which the queue's slack (kQueueSlots) covers.

struct WaveQueue {
    uint32_t* lq;
    int* tail_lds;      // ring tail in LDS: lanes may append from divergent code
    int head;           // wave-uniform ring head (only uniform code moves it)
    bool holding;       // wave-uniform: counted in *pending
    uint32_t* q;
    int* qhead;
    int* qtail;
    int* pending;
    uint32_t* lp;       // optional wave-local ring: items that never leave the wave
    int* ptail_lds;     // its tail in LDS
    int phead;          // wave-uniform head
    int* stall;         // watchdog word (nonzero: every wavefront exits)
    int budget;         // loop iterations this wavefront may make
    int ticket;         // per lane: shared-queue slot this lane waits on, or -1
    int iter;           // wave-uniform iteration counter
    int share_mask;     // hand-off polls every share_mask + 1 busy iterations
    int naps;           // wave-uniform idle back-off
    int hw;             // per lane: largest ring fill this lane has seen after a push

    // share_every (a power of two): busy iterations between polls for lanes
    // elsewhere that wait for work (rebalance).
    __device__ __forceinline__ void init(uint32_t* ring, int* ring_tail, uint32_t* gq,
                                         int* ctr_qhead, int* ctr_qtail, int* ctr_pending,
                                         int* ctr_stall, int step_budget,
                                         int share_every = kPollEvery,
                                         uint32_t* local_ring = nullptr,
                                         int* local_tail = nullptr) {
        lq = ring;
        tail_lds = ring_tail;
        lp = local_ring;
        ptail_lds = local_tail;
        phead = 0;
        if (lane_id() == 0) {
            *tail_lds = 0;
            if (ptail_lds) *ptail_lds = 0;
        }
        __builtin_amdgcn_wave_barrier();
        head = 0;
        holding = false;
        q = gq;
        qhead = ctr_qhead;
        qtail = ctr_qtail;
        pending = ctr_pending;
        stall = ctr_stall;
        budget = step_budget;
        ticket = -1;
        iter = 0;
        share_mask = share_every - 1;
        naps = 1;
        hw = 0;
    }

    __device__ __forceinline__ int tail() const {
        return __hip_atomic_load(tail_lds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    __device__ __forceinline__ int fill() const { return tail() - head; }

    // One item into the wave-local ring, from any lane, also from divergent
    // code.  Returns false (nothing pushed) when that ring is full.  Its items
    // are taken by idle lanes of this wave before any other work and never go
    // to the shared queue, so they need no room there.
    __device__ __forceinline__ bool push_local(uint32_t it) {
        int t = __hip_atomic_load(ptail_lds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        for (;;) {
            if (t - phead >= kLocalP) return false;
            if (__hip_atomic_compare_exchange_strong(ptail_lds, &t, t + 1, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WAVEFRONT)) {
                lp[t & (kLocalP - 1)] = it;
                return true;
            }
        }
    }

    // Idle lanes take items from the wave-local ring, then from the LDS ring.
    __device__ __forceinline__ void refill(uint32_t& item) {
        if (lp) {
            const uint64_t idle = ballot(item == kNone);
            const int avail =
                __hip_atomic_load(ptail_lds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) -
                phead;
            if (idle && avail > 0) {
                const int take = min(popc(idle), avail);
                const int rank = popc(idle & lanes_below());
                if (item == kNone && rank < take) item = lp[(phead + rank) & (kLocalP - 1)];
                phead += take;
            }
        }
        const uint64_t idle = ballot(item == kNone);
        const int avail = tail() - head;
        if (idle && avail > 0) {
            const int take = min(popc(idle), avail);
            const int rank = popc(idle & lanes_below());
            if (item == kNone && rank < take) item = lq[(head + rank) & (kLocalQ - 1)];
            head += take;
        }
    }

    // Idle lanes whose ticket slot has been filled take that item.
    __device__ __forceinline__ void resolve(uint32_t& item) {
        bool got = false;
        if (item == kNone && ticket >= 0) {
            const uint32_t x = (uint32_t)ld_dev((const int*)q + ticket);
            if (x != kNone) {
                st_dev((int*)q + ticket, (int)kNone);
                item = x;
                ticket = -1;
                got = true;
            }
        }
        const int r = popc(ballot(got));
        if (r) {
            if (lane_id() == 0) add_dev(pending, (holding ? 0 : 1) - r);
            holding = true;
        }
    }

    // Every lane takes a ticket (only when none is outstanding).
    __device__ __forceinline__ void claim() {
        int base = 0;
        if (lane_id() == 0) base = add_dev(qhead, kWave);
        ticket = __shfl(base, 0) + lane_id();
    }

    __device__ __forceinline__ void spill_ring(int k) {
        int base = 0;
        if (lane_id() == 0) {
            add_dev(pending, k);
            complete_mem();
            base = add_dev(qtail, k);
        }
        base = __shfl(base, 0);
        for (int i = lane_id(); i < k; i += kWave)
            st_dev((int*)q + base + i, (int)lq[(head + i) & (kLocalQ - 1)]);
        head += k;
    }

    // One item from any lane, also from divergent code: into the ring if it
    // has room, else straight to the shared queue.  The wave must be holding.
    __device__ __forceinline__ void push1(uint32_t it) {
        int t = tail();
        for (;;) {
            if (t - head >= kLocalQ) {
                add_dev(pending, 1);
                complete_mem();
                const int pos = add_dev(qtail, 1);
                st_dev((int*)q + pos, (int)it);
                return;
            }
            if (__hip_atomic_compare_exchange_strong(tail_lds, &t, t + 1, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WAVEFRONT)) {
                lq[t & (kLocalQ - 1)] = it;
                hw = max(hw, t + 1 - head);
                return;
            }
        }
    }

    // Append this lane's a and b (kNone = nothing), from uniform code: to the
    // ring, or to the shared queue when the ring has no room.
    __device__ __forceinline__ void push(uint32_t a, uint32_t b) {
        const uint64_t ma = ballot(a != kNone), mb = ballot(b != kNone);
        const int ca = popc(ma), total = ca + popc(mb);
        if (total == 0) return;
        const int ra = popc(ma & lanes_below());
        const int rb = ca + popc(mb & lanes_below());
        const int t = tail();
        if (total <= kLocalQ - (t - head)) {
            if (a != kNone) lq[(t + ra) & (kLocalQ - 1)] = a;
            if (b != kNone) lq[(t + rb) & (kLocalQ - 1)] = b;
            __builtin_amdgcn_wave_barrier();
            if (lane_id() == 0) *tail_lds = t + total;
            __builtin_amdgcn_wave_barrier();
            hw = max(hw, t + total - head);
            return;
        }
        int base = 0;
        if (lane_id() == 0) {
            add_dev(pending, total);
            complete_mem();
            base = add_dev(qtail, total);
        }
        base = __shfl(base, 0);
        if (a != kNone) st_dev((int*)q + base + ra, (int)a);
        if (b != kNone) st_dev((int*)q + base + rb, (int)b);
    }

    // Uniform code.  A ring close to full hands its oldest items above
    // kSpillAbove to the shared queue in one reservation (so single pushes
    // rarely take the slow path).  Now and then: if lanes elsewhere wait for
    // work (tickets beyond qtail), hand them part of the ring.
    __device__ __forceinline__ void rebalance() {
        if (fill() > kLocalQ - 256) {
            spill_ring(fill() - kSpillAbove);
            return;
        }
        if ((iter & share_mask) != 0) return;
        const int occ = fill();
        if (occ < 2) return;
        int waiting = 0;
        if (lane_id() == 0) waiting = ld_dev(qhead) - ld_dev(qtail);
        waiting = __shfl(waiting, 0);
        if (waiting > 0) spill_ring(min(occ / 2, waiting));
    }

    // Wave-uniform: true once some wavefront raised the stall word.
    __device__ __forceinline__ bool stalled() const {
        int s = 0;
        if (lane_id() == 0) s = ld_dev(stall);
        return __shfl(s, 0) != 0;
    }

    // Returns false when the whole computation is finished (or abandoned by
    // the watchdog).  Otherwise at least one lane of the wave holds an item.
    __device__ __forceinline__ bool acquire(uint32_t& item) {
        for (;;) {
            ++iter;
            if (iter > budget) {   // watchdog: give up, and make everyone else stop
                if (lane_id() == 0) st_dev(stall, 1);
                return false;
            }
            if ((iter & 255) == 0 && stalled()) return false;
            refill(item);
            const uint64_t busy = ballot(item != kNone);
            const bool tickets = ballot(ticket >= 0) != 0;
            if (busy) {
                naps = 1;
                if (busy != ~0ull && (iter & 15) == 0) {
                    if (tickets) resolve(item);
                    else if (tail() == head && (iter & (kPollEvery - 1)) == 0) claim();
                }
                return true;
            }
            if (holding) {
                if (lane_id() == 0) add_dev(pending, -1);
                holding = false;
            }
            if (!tickets) claim();
            resolve(item);
            if (ballot(item != kNone)) {
                naps = 1;
                return true;
            }
            if (ld_dev(pending) == 0 || stalled()) return false;
            for (int i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(127);
            naps = naps * 2 > kMaxNaps ? kMaxNaps : naps * 2;
        }
    }
};

// Block-wide maximum of a non-negative value; every thread gets the result.
__device__ __forceinline__ int block_max(int x, int* scratch) {
    for (int off = kWave / 2; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off));
    const int w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane_id() == 0) scratch[w] = x;
    __syncthreads();
    int m = 0;
    for (int i = 0; i < nw; ++i) m = max(m, scratch[i]);
    __syncthreads();
    return m;
}

// Block-wide sum; every thread gets the result.  `scratch` holds >= 16 words.
__device__ __forceinline__ uint64_t block_sum(uint64_t x, uint64_t* scratch) {
    x = wave_sum(x);
    const int w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane_id() == 0) scratch[w] = x;
    __syncthreads();
    uint64_t s = 0;
    for (int i = 0; i < nw; ++i) s += scratch[i];
    __syncthreads();
    return s;
}

// After a call abandoned by the watchdog, items and consumed tickets may be
// left in the shared queue.  The output kernel that follows the persistent
// one restores every slot to kNone (grid-stride), so the next call starts
// from a clean queue; when nothing stalled it only reads the stall word.
__device__ __forceinline__ void clear_queue_if_stalled(const int* ctr, uint32_t* q,
                                                       long long qwords) {
    if (!q || ld_dev(ctr + kStall) == 0) return;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < qwords;
         i += (long long)gridDim.x * blockDim.x)
        q[i] = kNone;
}

// ------------------------------------------------------------ graph views
// A view gives, for vertex v: the cursor range [begin(v), end(v)) and the
// target of cursor position p.  `vctx` carries a per-vertex value the view
// needs (the first vertex of v's graph for packed batches).
// The CSR arrays are read with non-temporal loads: they are streamed once by
// the first sweep, and caching them would evict the list heads and records
// that the propagation keeps revisiting.
struct ExplicitView {
    const int* row_off;
    const int* col;
    __device__ __forceinline__ int vctx(int) const { return 0; }
    __device__ __forceinline__ int begin(int v) const { return __builtin_nontemporal_load(row_off + v); }
    __device__ __forceinline__ int end(int v) const { return __builtin_nontemporal_load(row_off + v + 1); }
    __device__ __forceinline__ int target(int, int p, int) const { return __builtin_nontemporal_load(col + p); }
};

// SplitMix64 finalizer (Steele, Lea, Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr uint64_t kTagZero = 0x5A45524F00000000ull;
constexpr uint64_t kTagDeg = 0x4445470000000000ull;
constexpr uint64_t kTagNbr = 0x4E42520000000000ull;

// Hash-generated graph: no stored edges; cursor positions are successor indices.
struct ImplicitView {
    uint64_t seed;
    uint64_t zero_thr;
    const uint64_t* table;   // 256 thresholds, normally staged in LDS
    uint32_t mask;           // n - 1
    __device__ __forceinline__ int vctx(int) const { return 0; }
    __device__ __forceinline__ int begin(int) const { return 0; }
    __device__ __forceinline__ int end(int v) const {
        uint64_t key = (uint64_t)(uint32_t)v << 8;
        if (mix64(seed ^ kTagZero ^ key) < zero_thr) return 0;
        uint64_t u = mix64(seed ^ kTagDeg ^ key);
        // 1 + #{j < 255 : u >= table[j]}; table is non-decreasing
        int lo = 0, hi = 255;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (u >= table[mid]) lo = mid + 1; else hi = mid;
        }
        return 1 + lo;
    }
    __device__ __forceinline__ int target(int v, int p, int) const {
        uint64_t key = ((uint64_t)(uint32_t)v << 8) | (uint32_t)p;
        return (int)(mix64(seed ^ kTagNbr ^ key) & mask);
    }
};

// Packed batch: graph-local targets shifted by the first vertex of the
// source's graph, held per vertex in `base` (filled once per call).
struct BatchView {
    const int* row_off;
    const int* col;
    const int* base;
    __device__ __forceinline__ int vctx(int v) const { return base[v]; }
    __device__ __forceinline__ int begin(int v) const { return row_off[v]; }
    __device__ __forceinline__ int end(int v) const { return row_off[v + 1]; }
    __device__ __forceinline__ int target(int, int p, int b) const { return b + col[p]; }
};

}  // namespace trim
