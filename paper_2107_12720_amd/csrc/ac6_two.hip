// ac6_two.hip -- two-sided AC-6 trimming on gfx950: the in-degree check of
// Section 4.1 (with G^T in memory, a vertex must also keep a live
// predecessor) applied to the AC-6-based algorithm (Section 6.2).
//
// A vertex stays only while it has a live successor and a live predecessor.
// It keeps one support per side, each found by the AC-6 support search over
// its own list: successors in G for the out-side, predecessors in G^T for the
// in-side.  Each side has the list pair and records of the one-sided kernels
// (ac6.hip):
//   hout[2w], hout[2w+1]  S_more / S_last of the vertices whose out-support is w
//   hin[2w],  hin[2w+1]   the same for the vertices whose in-support is w
//   rec_out[v], rec_in[v] (next, cursor) of v in the list of its support
// Removing x exchanges both pairs of x with kDead (one 8-byte exchange each).
// That hands back the predecessors x supported (they resume their out-scans)
// and the successors x supported (in-scans); members of an S_last list lose
// their last neighbour on that side and are removed at once.  Each pair is a
// lock of its own, as in the one-sided algorithm: its first exchange takes the
// lists, a later one (a vertex removed from both sides at once) gets kDead.
//
// A vertex removed through one side may still be a member of a list on the
// other side.  When that list is handed back the member is skipped (no scan)
// and the walk goes on to the next member.  A member that dies during its own
// scan may still join a list; it is skipped when that list is handed back.
//
// Checks per vertex: a live vertex ends with each support at its first
// finally-live neighbour, so its checks do not depend on the schedule; a
// removed one checks at most its two lists once, and at least the whole list
// of the side that removed it.
//
// Kernels, in stream order: ac6t_init (list heads, the bitmap of vertices
// without successors or predecessors, counters), ac6t_sweep (both support
// searches per vertex; only that bitmap's vertices are removed while it runs,
// so joining is a plain exchange), ac6_jump (the forest collapse of the
// one-sided kernels over the out-side S_last links; the default, off with
// TRIM_FLAG_STEPWISE: a chain that ends in a vertex without successors falls
// in O(log length) rounds instead of one removal after another),
// ac6t_propagate (persistent workers on per-wavefront LDS rings), pack.
#include "trim_device.h"
#include "trim_stats.h"
#include "trim_internal.h"
#include "ac6_support.h"
#include "scc_internal.h"
#include "forest_jump.h"

namespace trim {

namespace {

struct TwoGraph {
    const int* row_off;
    const int* col;
    const int* rrow_off;
    const int* rcol;
    int* hout;
    int* hin;
    uint64_t* rec_out;
    uint64_t* rec_in;
    int* ext;   // out-side split S_more heads (ac6_support.h), or nullptr
};

// Sets dead0 bit v iff v has no successor, no predecessor, or is preset
// (removed before trimming); each wavefront covers 64 consecutive ids (the
// last may write one word past ceil(n/32), which the buffer has).
__global__ void ac6t_init(TwoGraph g, int n, uint32_t* dead0, const uint32_t* preset, int* ctr,
                          uint64_t* worker_edges, int P, trim_stats_t* stats) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < kCtrInts) ctr[tid] = 0;
    for (int p = tid; p < P; p += gridDim.x * blockDim.x) worker_edges[p] = 0;
    if (stats && tid < (int)(sizeof(trim_stats_t) / 8)) ((uint64_t*)stats)[tid] = 0;
    for (int v = tid; v < n; v += gridDim.x * blockDim.x) {
        const bool d = g.row_off[v + 1] == g.row_off[v] || g.rrow_off[v + 1] == g.rrow_off[v] ||
                       (preset && ((preset[v >> 5] >> (v & 31)) & 1u));
        const int h = d ? kDead : kEmpty;
        reinterpret_cast<int2*>(g.hout)[v] = make_int2(h, h);
        if (g.ext)
            for (int j = 0; j < kMoreLists - 1; ++j) g.ext[(kMoreLists - 1) * (long long)v + j] = h;
        reinterpret_cast<int2*>(g.hin)[v] = make_int2(h, h);
        const uint64_t m = ballot(d);
        if (lane_id() == 0) {
            dead0[v >> 5] = (uint32_t)m;
            dead0[(v >> 5) + 1] = (uint32_t)(m >> 32);
        }
    }
}

__device__ __forceinline__ bool bit(const uint32_t* bm, int v) { return (bm[v >> 5] >> (v & 31)) & 1u; }

constexpr int kTSweepUnroll = 4;   // vertices per lane in flight in the first sweep
// entries buffered in LDS before one shared append: room for one step of the
// largest workgroup (1,024 lanes x kTSweepUnroll)
constexpr int kCasBuf = 1024 * kTSweepUnroll;
// In-side joins of one sweep step are combined per list in an LDS table
// (open addressing, kJoinProbes probes): a G^T list in source order makes a
// hub the first predecessor of many of its successors, and on R-MAT scale 22
// one list would otherwise take about 96,000 exchanges, serialised at its
// address.  A full table only sends a join to the list directly.
constexpr int kJoinLog = 10;
constexpr int kJoinTable = 1 << kJoinLog;
constexpr int kJoinProbes = 8;
constexpr int kNoChain = -0x7FFFFFFF - 1;   // first joiner of a chain (no LDS predecessor)

// The first sweep: for every vertex v outside dead0, the first successor
// outside dead0 (its out-support) and, only if there is one, the first
// predecessor outside dead0 (its in-support), each joined by exchange; v is a
// casualty if either is missing.  Only dead0's vertices are removed while
// this kernel runs, so a neighbour is live iff its dead0 bit is clear.
//
// Each lane keeps kTSweepUnroll vertices in flight, blockDim apart: their
// offsets on both sides, then their first successors and first predecessors
// and those neighbours' dead0 bits, then their joins, are issued before any
// result is waited for.  The in-side loads are issued whatever the out-side
// finds (a load is no check); the in-side scan past dead0 and the in-side
// join happen only for a vertex that found its out-support, so the checks
// counted are those of the one-vertex-at-a-time reading.
//
// With jp (the forest collapse over the out-side S_last links, forest_jump.h):
// jp[v] = v's out-support if that is v's last successor and v keeps an
// in-support (a tree member, listed in jlist), ~v if v found no live
// successor or no live predecessor (a removed root, listed with kRootBit),
// v itself otherwise.  Without jp, the vertices that found none are queued as
// close items.
__global__ void ac6t_sweep(TwoGraph g, int n, int chunk, const uint32_t* dead0, uint32_t* q,
                           int* ctr, uint64_t* worker_edges, int P, uint64_t* part, int sched,
                           int* jp, uint32_t* jlist) {
    constexpr int U = kTSweepUnroll;
    __shared__ uint32_t cas[kCasBuf];
    __shared__ int tkey[kJoinTable], thead[kJoinTable];
    __shared__ int s_chunk, s_ncas, s_base;
    __shared__ uint64_t red[16];
    if (threadIdx.x == 0) s_ncas = 0;
    for (int i = threadIdx.x; i < kJoinTable; i += blockDim.x) {
        tkey[i] = -1;
        thead[i] = kNoChain;
    }
    uint64_t edges = 0, degsum = 0;
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
        if (threadIdx.x == 0) s_chunk = add_dev(ctr + kCursor, chunk);
        __syncthreads();
        const int claim = s_chunk;
        __syncthreads();
        if (claim >= n) break;
        int cb = claim;
        if (sched & TRIM_SCHED_REVERSE) cb = ((n + chunk - 1) / chunk - 1 - claim / chunk) * chunk;
        const int ce = cb + chunk < n ? cb + chunk : n;
        for (int base = cb; base < ce; base += U * blockDim.x) {
            int v[U], b[U], e[U], rb[U], re[U], po[U], pi[U], wo[U], wi[U];
            bool live[U], oko[U], oki[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                v[k] = base + k * blockDim.x + threadIdx.x;
                b[k] = e[k] = rb[k] = re[k] = 0;
                if (v[k] < ce) {
                    b[k] = g.row_off[v[k]];
                    e[k] = g.row_off[v[k] + 1];
                    rb[k] = g.rrow_off[v[k]];
                    re[k] = g.rrow_off[v[k] + 1];
                }
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                degsum += (uint64_t)(e[k] - b[k]);
                // dead0 holds every vertex without successors or predecessors
                live[k] = v[k] < ce && !bit(dead0, v[k]);
                po[k] = b[k];
                pi[k] = rb[k];
                wo[k] = wi[k] = 0;
                if (b[k] < e[k]) wo[k] = __builtin_nontemporal_load(g.col + b[k]);
                if (rb[k] < re[k]) wi[k] = __builtin_nontemporal_load(g.rcol + rb[k]);
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                oko[k] = live[k] && !bit(dead0, wo[k]);
                oki[k] = live[k] && !bit(dead0, wi[k]);
            }
            // the rare serial scans past dead0
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (live[k] && !oko[k]) {
                    for (++po[k]; po[k] < e[k]; ++po[k]) {
                        wo[k] = __builtin_nontemporal_load(g.col + po[k]);
                        if (!bit(dead0, wo[k])) break;
                    }
                    oko[k] = po[k] < e[k];
                }
                if (oko[k] && !oki[k]) {
                    for (++pi[k]; pi[k] < re[k]; ++pi[k]) {
                        wi[k] = __builtin_nontemporal_load(g.rcol + pi[k]);
                        if (!bit(dead0, wi[k])) break;
                    }
                    oki[k] = pi[k] < re[k];
                }
            }
            int oldo[U], oldi[U], key[U], hs[U];
            bool lead[U];
            // out-side joins first: their round trips overlap the in-side
            // combining below
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (oko[k]) {
                    if (sched & TRIM_SCHED_JITTER)
                        jitter_nap(((uint64_t)blockIdx.x << 32) ^ (uint32_t)v[k]);
                    oldo[k] = xchg_dev(join_slot(g.hout, g.ext, wo[k], po[k] + 1 == e[k], v[k]),
                                       v[k]);
                }
            }
            // in-side joins, step 1: join the workgroup's chain for the list
            // (a free or matching table entry within kJoinProbes probes; else
            // the list directly)
#pragma unroll
            for (int k = 0; k < U; ++k) {
                hs[k] = -1;
                lead[k] = false;
                if (oko[k] && oki[k]) {
                    key[k] = 2 * wi[k] + (pi[k] + 1 == re[k]);
                    uint32_t h = ((uint32_t)key[k] * 0x9E3779B1u) >> (32 - kJoinLog);
                    for (int t = 0; t < kJoinProbes; ++t, h = (h + 1) & (kJoinTable - 1)) {
                        const int cur = atomicCAS(&tkey[h], -1, key[k]);
                        if (cur == -1 || cur == key[k]) {
                            lead[k] = cur == -1;
                            hs[k] = (int)h;
                            oldi[k] = atomicExch(&thead[h], v[k]);
                            break;
                        }
                    }
                    if (hs[k] < 0) {
                        if (sched & TRIM_SCHED_JITTER)
                            jitter_nap((((uint64_t)blockIdx.x << 32) ^ (uint32_t)v[k]) ^ 1);
                        oldi[k] = xchg_dev(g.hin + key[k], v[k]);
                    }
                }
            }
            __syncthreads();
            // step 2: one exchange per list publishes the whole chain; the
            // list's previous head goes where the chain's head was
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (lead[k]) {
                    if (sched & TRIM_SCHED_JITTER)
                        jitter_nap((((uint64_t)blockIdx.x << 32) ^ (uint32_t)v[k]) ^ 1);
                    thead[hs[k]] = xchg_dev(g.hin + key[k], thead[hs[k]]);
                }
            }
            __syncthreads();
            // step 3: the chain's first joiner links to the previous head
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (hs[k] >= 0 && oldi[k] == kNoChain) oldi[k] = thead[hs[k]];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (lead[k]) {
                    tkey[hs[k]] = -1;
                    thead[hs[k]] = kNoChain;
                }
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                bool casualty = false, member = false;
                if (live[k]) {
                    if (oko[k]) {
                        g.rec_out[v[k]] = pack_rec(oldo[k], po[k]);
                        edges += (uint64_t)(po[k] - b[k] + 1);
                        if (oki[k]) {
                            g.rec_in[v[k]] = pack_rec(oldi[k], pi[k]);
                            edges += (uint64_t)(pi[k] - rb[k] + 1);
                        } else {
                            edges += (uint64_t)(re[k] - rb[k]);
                        }
                    } else {
                        edges += (uint64_t)(e[k] - b[k]);
                    }
                    casualty = !(oko[k] && oki[k]);
                    if (jp) {
                        member = !casualty && po[k] + 1 == e[k];
                        jp[v[k]] = casualty ? ~v[k] : member ? wo[k] : v[k];
                    }
                }
                const bool put = casualty || member;
                const uint64_t mask = ballot(put);
                if (mask) {
                    int wbase = 0;
                    if (lane_id() == 0) wbase = atomicAdd(&s_ncas, popc(mask));
                    wbase = __shfl(wbase, 0);
                    if (put)
                        cas[wbase + popc(mask & lanes_below())] =
                            (uint32_t)v[k] | (jp && casualty ? kRootBit : 0u);
                }
            }
            __syncthreads();
            if (s_ncas > kCasBuf - U * (int)blockDim.x) flush();
        }
    }
    flush();
    edges = block_sum(edges, red);
    degsum = block_sum(degsum, red);
    if (threadIdx.x == 0) {
        if (edges) add_dev(worker_edges + (blockIdx.x % P), edges);
        part[kPartSweep * kPartStride + blockIdx.x] = edges;
        part[kPartDeg * kPartStride + blockIdx.x] = degsum;
    }
}

// Work items: a 3-bit kind above a 29-bit vertex id (n <= 2^29).
//   CLOSE(x)        x lost every neighbour on one side: close both pairs of x;
//   LAST_OUT(x)     x is a member of a closed S_last list on the out-side (its
//                   last successor died): remove it; rec_out[x] links to the
//                   next member;  LAST_IN(x) the same on the in-side;
//   MORE_OUT(x)     x heads (the rest of) a closed S_more list on the
//                   out-side: follow the links and hand each member out as a
//                   RESCAN_OUT item, up to kTWalk members in a row;
//                   MORE_IN(x) likewise on the in-side;
//   RESCAN_OUT(x)   resume x's out-scan after its old support, unless x is
//                   already removed;  RESCAN_IN(x) likewise on the in-side.
// The walk only loads links, one memory round trip per member, so a hub's
// long list is not walked at the pace of its members' scans: the rescans go
// to the wave-local ring, where the other lanes of the walking wave take
// them (never to the shared queue, whose room is counted per vertex).
enum : uint32_t {
    kTClose = 0, kTLastOut = 1, kTLastIn = 2, kTMoreOut = 3, kTMoreIn = 4, kTRescanOut = 5,
    kTRescanIn = 6
};
constexpr int kTWalk = 32;   // S_more members one MORE item hands out in a row
constexpr uint32_t kTIdMask = 0x1FFFFFFFu;
__device__ __forceinline__ uint32_t titem(uint32_t kind, int v) { return (kind << 29) | (uint32_t)v; }
__device__ __forceinline__ uint32_t last_kind(int side) { return side ? kTLastIn : kTLastOut; }
constexpr int kTHops = 256;   // removals one item may chain in a row
// Busy iterations between polls for waiting lanes elsewhere: 16, as for the
// one-sided explicit view (measured at 512 workers: the 65,536-vertex
// core+tail graph's propagation about 20 % faster than with 64, the R-MAT 22
// graphs with and without the chain unchanged).
constexpr int kTShareEvery = 16;

__global__ __launch_bounds__(256) void ac6t_propagate(TwoGraph g, uint32_t* q, int* ctr,
                                                      uint64_t* worker_edges, uint64_t* part,
                                                      int sched, int budget) {
    __shared__ uint32_t rings[256 / kWave][kLocalQ];
    __shared__ int ring_tail[256 / kWave];
    __shared__ uint32_t local_rings[256 / kWave][kLocalP];
    __shared__ int local_tail[256 / kWave];
    __shared__ uint64_t red[16];
    WaveQueue wq;
    const int wv = threadIdx.x / kWave;
    wq.init(rings[wv], &ring_tail[wv], q, ctr + kQHead, ctr + kQTail, ctr + kPending,
            ctr + kStall, budget, kTShareEvery, local_rings[wv], &local_tail[wv]);
    const ExplicitView out_view{g.row_off, g.col}, in_view{g.rrow_off, g.rcol};
    uint32_t item = kNone;
    uint64_t edges = 0, closes = 0, joins = 0, visited = 0;
    while (wq.acquire(item)) {
        uint32_t keep = kNone;
        bool close_now = false;
        int cx = 0;
        int side = -1;   // list of cx's S_last membership: 0 out, 1 in, -1 none
        if (item != kNone) {
            const int x = (int)(item & kTIdMask);
            const uint32_t kind = item >> 29;
            if (kind >= kTMoreOut) {
                const bool in = kind == kTMoreIn || kind == kTRescanIn;
                uint64_t* rec = in ? g.rec_in : g.rec_out;
                const uint32_t walk = in ? kTMoreIn : kTMoreOut;
                int rx = -1, cont = -1;   // a member rescanned by this lane now; the rest
                if (kind <= kTMoreIn) {
                    // Each link is read before its member is handed out (a
                    // rescan that re-joins rewrites the member's record).  The
                    // last member of a burst, and any member the full local
                    // ring does not take, is rescanned by the walker itself.
                    int y = x;
                    for (int h = 0;; ++h) {
                        const int ny = ld_dev(rec_link(rec, y));
                        visited += 1;
                        if (h + 1 < kTWalk &&
                            wq.push_local(titem(in ? kTRescanIn : kTRescanOut, y))) {
                            if (ny < 0) break;
                            y = ny;
                            continue;
                        }
                        rx = y;
                        cont = ny;
                        break;
                    }
                } else {
                    rx = x;
                }
                if (rx >= 0) {
                    // rx is in no list of this side until it joins again: its
                    // record is stable
                    const uint64_t r = ld_dev(rec + rx);
                    bool stays = true;   // a removed member is skipped
                    if (ld_dev(g.hout + 2 * rx) != kDead) {
                        if (sched & TRIM_SCHED_JITTER) jitter_nap(rx);
                        stays = in ? resume(in_view, rx, rec_cursor(r) + 1, g.hin, g.rec_in, edges,
                                            sched)
                                   : resume(out_view, rx, rec_cursor(r) + 1, g.hout, g.rec_out,
                                            edges, sched, g.ext);
                        joins += stays;
                    }
                    if (stays) {
                        if (cont >= 0) keep = titem(walk, cont);
                    } else {
                        if (cont >= 0) wq.push1(titem(walk, cont));
                        close_now = true;
                        cx = rx;
                    }
                }
            } else {
                close_now = true;
                cx = x;
                side = kind == kTLastOut ? 0 : kind == kTLastIn ? 1 : -1;
            }
        }
        if (close_now) {
            // Close cx and go on depth first: into S_last on the out-side, else
            // on the in-side, else to the next member of cx's own S_last list.
            // One step = the two pair exchanges plus, for a list member, the
            // load of its link, all in flight together; the next step's memory
            // operations are issued before this step's pushes.
            int link = side >= 0 ? ld_dev(rec_link(side ? g.rec_in : g.rec_out, cx)) : -1;
            ClosedLists o = close_lists(g.hout, g.ext, cx);
            int2 i = xchg2_dev(g.hin + 2 * cx, kDead, kDead);
            int fill = 0;
            for (int hop = 0;; ++hop) {
                closes += (o.more[0] != kDead);   // the out-pair's exchange counts the removal
                const ClosedLists co = o;
                const int bo = co.last, ai = i.x, bi = i.y;
                const int sib = side >= 0 ? link : -1;
                int next = sib, nside = side;
                if (bo >= 0) {
                    next = bo;
                    nside = 0;
                } else if (bi >= 0) {
                    next = bi;
                    nside = 1;
                }
                visited += (bo >= 0) + (bi >= 0) + (sib >= 0);
                const bool go = next >= 0 && hop + 1 < kTHops && fill <= kLocalQ - 256;
                if (go) {
                    if (sched & TRIM_SCHED_JITTER) jitter_nap(((uint64_t)next << 8) ^ hop);
                    link = ld_dev(rec_link(nside ? g.rec_in : g.rec_out, next));
                    o = close_lists(g.hout, g.ext, next);
                    i = xchg2_dev(g.hin + 2 * next, kDead, kDead);
                }
#pragma unroll
                for (int j = 0; j < kMoreLists; ++j)
                    if (co.more[j] >= 0) wq.push1(titem(kTMoreOut, co.more[j]));
                if (ai >= 0) wq.push1(titem(kTMoreIn, ai));
                if (bo >= 0 && bi >= 0) wq.push1(titem(kTLastIn, bi));
                if ((bo >= 0 || bi >= 0) && sib >= 0) wq.push1(titem(last_kind(side), sib));
                fill = wq.fill();
                if (!go) {
                    if (next >= 0) keep = titem(last_kind(nside), next);
                    break;
                }
                side = nside;
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

// The forest collapse's removal (forest_jump.h): every list head of v
// exchanged with kDead; its out-side and in-side S_more lists go back to the
// propagation as walks, and its in-side S_last list as a chain of removals.
// (Its out-side S_last members are its own tree's, removed by the same
// rounds.)
static_assert(kJumpItems >= kMoreLists + 2, "a two-sided removal hands back its S_more lists "
                                            "and both in-side lists");
struct TwoSidedKill {
    int* hout;
    int* hin;
    int* ext;
    __device__ __forceinline__ void operator()(int v, uint32_t (&item)[kJumpItems]) const {
        const ClosedLists o = close_lists(hout, ext, v);
        const int2 i = xchg2_dev(hin + 2 * v, kDead, kDead);
#pragma unroll
        for (int j = 0; j < kMoreLists; ++j)
            if (o.more[j] >= 0) item[j] = titem(kTMoreOut, o.more[j]);
        if (i.x >= 0) item[kMoreLists] = titem(kTMoreIn, i.x);
        if (i.y >= 0) item[kMoreLists + 1] = titem(kTLastIn, i.y);
    }
};

// Live bitmap by ballot, plus the checks the live vertices made, read off
// their final cursors: a live vertex's supports end at its first finally-live
// successor and predecessor, so it checked fl_out + 1 + fl_in + 1 positions
// whatever the schedule.  Restores the shared queue after a stalled call.
__global__ void ac6t_pack(TwoGraph g, int n, uint32_t* bitmap, uint64_t* part, const int* ctr,
                          uint32_t* q, long long qwords) {
    __shared__ uint64_t red[16];
    clear_queue_if_stalled(ctr, q, qwords);
    const int nwords = (n + 31) >> 5;
    const int waves = (gridDim.x * blockDim.x) / kWave;
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    uint64_t live_cnt = 0, live_edges = 0;
    for (int base = wid * kWave; base < n; base += waves * kWave) {
        const int v = base + lane_id();
        const bool live = v < n && g.hout[2 * v] != kDead;
        if (live)
            live_edges += (uint64_t)(rec_cursor(g.rec_out[v]) - g.row_off[v] + 1) +
                          (uint64_t)(rec_cursor(g.rec_in[v]) - g.rrow_off[v] + 1);
        const uint64_t b = ballot(live);
        if (lane_id() == 0) {
            const int w = base >> 5;
            bitmap[w] = (uint32_t)b;
            if (w + 1 < nwords) bitmap[w + 1] = (uint32_t)(b >> 32);
            live_cnt += (uint64_t)popc(b);
        }
    }
    live_cnt = block_sum(live_cnt, red);
    live_edges = block_sum(live_edges, red);
    if (threadIdx.x == 0) {
        part[kPartLive * kPartStride + blockIdx.x] = live_cnt;
        part[kPartLiveEdges * kPartStride + blockIdx.x] = live_edges;
    }
}

inline int grid_for(long long n, int block, int max_blocks = 1 << 20) {
    long long b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

}  // namespace

hipError_t ac6_two_csr(const trim_csr_t& gc, const Work& w, const Work2& x, const LaunchCfg& lc,
                       uint32_t* bitmap, uint64_t* worker_edges, trim_stats_t* stats) {
    return ac6_two_csr_preset(gc, w, x, lc, bitmap, worker_edges, stats, nullptr);
}

hipError_t ac6_two_csr_preset(const trim_csr_t& gc, const Work& w, const Work2& x,
                              const LaunchCfg& lc, uint32_t* bitmap, uint64_t* worker_edges,
                              trim_stats_t* stats, const uint32_t* preset) {
    const int n = gc.n, P = lc.workers, B = lc.block;
    // split out-side S_more lists where their heads exist and the shared
    // queue has room for the items a close then hands back
    const bool split = w.ext && n <= kSplitMaxN &&
                       x.qwords >= (long long)kQueuePerVertexTwoSplit * n + kQueueSlots;
    TwoGraph g{gc.row_off, gc.col, gc.rrow_off, gc.rcol, w.a, x.hin, w.b, x.rec_in,
               split ? w.ext : nullptr};
    uint32_t* dead0 = reinterpret_cast<uint32_t*>(w.c);
    int sweep_blocks = 0, pack_blocks = 0;
    {
        Timed t(lc, "ac6t_init");
        hipLaunchKernelGGL(ac6t_init, dim3(grid_for(n, 256, 16384)), dim3(256), 0, lc.stream, g,
                           n, dead0, preset, w.ctr, worker_edges, P, stats);
    }
    if (n > 0) {
        const int chunk = sweep_chunk(lc, n, B);
        sweep_blocks = grid_for(n, chunk, lc.cus * 8);
        {
            Timed t(lc, "ac6t_sweep");
            hipLaunchKernelGGL(ac6t_sweep, dim3(sweep_blocks), dim3(B), 0, lc.stream, g, n, chunk,
                               dead0, x.q, w.ctr, worker_edges, P, w.part, lc.schedule,
                               lc.forest ? w.jp : nullptr, lc.forest ? w.e : nullptr);
        }
        if (lc.forest) {
            Timed t(lc, "ac6t_jump");
            hipLaunchKernelGGL(ac6_jump<TwoSidedKill>, dim3(phase_blocks(n, lc.cus)), dim3(256), 0,
                               lc.stream, TwoSidedKill{g.hout, g.hin, g.ext}, w.jp, w.e, w.e + n, x.q,
                               w.ctr, jump_rounds(n), lc.budget);
        }
        {
            Timed t(lc, "ac6t_propagate");
            hipLaunchKernelGGL(ac6t_propagate, dim3(P), dim3(256), 0, lc.stream, g, x.q, w.ctr,
                               worker_edges, w.part, lc.schedule, lc.budget);
        }
        Timed t(lc, "ac6t_pack");
        pack_blocks = grid_for(n, 256, lc.cus * 4);
        hipLaunchKernelGGL(ac6t_pack, dim3(pack_blocks), dim3(256), 0, lc.stream, g, n, bitmap,
                           w.part, w.ctr, x.q, x.qwords);
    }
    if (stats) {
        Timed t(lc, "finalize");
        hipLaunchKernelGGL(finalize_stats, dim3(1), dim3(1024), 0, lc.stream, n, P, sweep_blocks,
                           n > 0 ? P : 0, pack_blocks, n > 0 ? P : 0, worker_edges, w.part,
                           w.ctr, stats, 0, pack_blocks);
    }
    return hipGetLastError();
}

int ac6_two_max_workers_per_cu(int) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ac6t_propagate, 256, 0) != hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

}  // namespace trim
