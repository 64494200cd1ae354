// ac3.hip -- AC-3-based graph trimming on gfx950 (Section 4.1, Alg. TraditionalTrim).
//
// Repetitions ("rounds") of a sweep over the live vertices, until a round
// removes nothing.  Each vertex keeps the edge_index cursor of Section 8:
// successors found DEAD are passed for good, the first successor that is not
// DEAD ends the scan and is checked again in the next round.
//
// A round reads the statuses as they were at its start: dround[w] holds the
// round in which w was removed (INT_MAX while live), and w counts as DEAD in
// round r iff dround[w] < r.  A removal in round r is therefore seen from
// round r+1 on, whatever the lane order, which makes the result of every round
// and the number of rounds (alpha + 1, Def. of alpha) deterministic.
//
// All rounds run inside one cooperative launch: the live vertices of round r
// sit in a compacted list, survivors are appended (wavefront-aggregated) to
// the list of round r+1, and a grid barrier separates rounds.  List sizes
// rotate over three counter slots so that resetting the slot of round r+2
// never races with readers of rounds r and r+1.
//
// Two-sided rounds (a vertex must also keep a live predecessor, Section 4.1)
// are ac3_init2 / ac3_rounds2 below: a second cursor over G^T, checked after
// the successor cursor.
#include <climits>

#include "trim_device.h"
#include "trim_stats.h"
#include "trim_internal.h"
#include "block_append.h"
#include "grid_barrier.h"

namespace trim {

namespace {

template <class View>
struct Stage3 {
    static constexpr int kWords = 1;
    __device__ static void apply(View&, uint64_t*) {}
};
template <>
struct Stage3<ImplicitView> {
    static constexpr int kWords = 256;
    __device__ static void apply(ImplicitView& g, uint64_t* lds) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) lds[i] = g.table[i];
        __syncthreads();
        g.table = lds;
    }
};

// A list of live vertices holds, per entry, the vertex and the target of its
// cursor (kNoTarget without successors), as two arrays of `n` ints.
constexpr int kNoTarget = -1;

// With a preset bitmap (vertices removed before trimming, the vertex sampling
// of Section 9) those vertices get removal round 0, so every round reads them
// as DEAD, and the first list is built by ac3_list_preset without them.
template <class View>
__global__ void ac3_init(View g, int n, const uint32_t* preset, int* ptr, int* dround,
                         int* list1, int* ctr, uint64_t* worker_edges, int P,
                         trim_stats_t* stats) {
    __shared__ uint64_t lds[Stage3<View>::kWords];
    Stage3<View>::apply(g, lds);
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < kCtrInts) ctr[tid] = (tid == kCnt0 + 1 && !preset) ? n : 0;
    for (int p = tid; p < P; p += gridDim.x * blockDim.x) worker_edges[p] = 0;
    if (stats && tid < (int)(sizeof(trim_stats_t) / 8)) ((uint64_t*)stats)[tid] = 0;
    for (int v = tid; v < n; v += gridDim.x * blockDim.x) {
        const int b = g.begin(v), e = g.end(v);
        ptr[v] = b;
        if (preset) {
            dround[v] = ((preset[v >> 5] >> (v & 31)) & 1u) ? 0 : INT_MAX;
        } else {
            dround[v] = INT_MAX;
            list1[v] = v;
            list1[n + v] = b < e ? g.target(v, b, g.vctx(v)) : kNoTarget;
        }
    }
}

// The first list without the preset vertices (one reservation per block and
// step; the order of the list does not matter to the rounds).
template <class View>
__global__ void ac3_list_preset(View g, int n, const uint32_t* preset, int* list1, int* ctr) {
    __shared__ uint64_t lds[Stage3<View>::kWords];
    __shared__ int s_wave[1024 / kWave], s_base;
    Stage3<View>::apply(g, lds);
    const int step = gridDim.x * blockDim.x * 4;
    for (int base = blockIdx.x * blockDim.x * 4; base < n; base += step) {
        int v[4], c = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = base + j * blockDim.x + threadIdx.x;
            const bool keep = x < n && !((preset[x >> 5] >> (x & 31)) & 1u);
            v[j] = keep ? x : -1;
            c += keep;
        }
        int slot = block_append_base(c, ctr + kCnt0 + 1, nullptr, s_wave, &s_base);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (v[j] < 0) continue;
            const int b = g.begin(v[j]), e = g.end(v[j]);
            list1[slot] = v[j];
            list1[n + slot] = b < e ? g.target(v[j], b, g.vctx(v[j])) : kNoTarget;
            ++slot;
        }
    }
}

// kUnroll list entries per lane per step, their loads in flight together, and
// one output reservation per workgroup per step (a reservation per wavefront
// made the list counter a single-address hot spot: thousands of serialised
// atomics per round).  An entry whose cursor target
// is still live costs one random access (the target's removal round); only
// when it has died are the cursor, the offsets and further successors read.
constexpr int kUnroll = 4;

template <class View>
__global__ __launch_bounds__(256) void ac3_rounds(View g, int n, int* ptr, int* dround,
                                                  int* list0, int* list1, int* ctr,
                                                  uint64_t* worker_edges, trim_stats_t* stats,
                                                  int budget) {
    __shared__ uint64_t lds[Stage3<View>::kWords];
    __shared__ int s_wave[256 / kWave], s_base;
    Stage3<View>::apply(g, lds);
    uint64_t edges = 0;
    int r = 1;
    const int stride = gridDim.x * blockDim.x;
    for (;; ++r) {
        const int* in = (r & 1) ? list1 : list0;
        int* out = (r & 1) ? list0 : list1;
        const int cnt_in = ld_dev(ctr + kCnt0 + r % 3);
        int* cnt_out = ctr + kCnt0 + (r + 1) % 3;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st_dev(ctr + kCnt0 + (r + 2) % 3, 0);
            add_dev(ctr + kAcWork, cnt_in);
        }
        for (int base = blockIdx.x * blockDim.x; base < cnt_in; base += stride * kUnroll) {
            int v[kUnroll], w[kUnroll], d[kUnroll];
            bool keep[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                const int i = base + k * stride + threadIdx.x;
                v[k] = -1;
                if (i < cnt_in) {
                    v[k] = ld_dev(in + i);
                    w[k] = ld_dev(in + n + i);
                }
            }
#pragma unroll
            for (int k = 0; k < kUnroll; ++k)
                d[k] = (v[k] >= 0 && w[k] != kNoTarget) ? ld_dev(dround + w[k]) : 0;
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                keep[k] = false;
                if (v[k] < 0) continue;
                if (w[k] != kNoTarget && d[k] >= r) {   // the cursor edge, checked again
                    edges += 1;
                    keep[k] = true;
                    continue;
                }
                // the cursor target is removed (or there is none): scan on
                const int p0 = ld_dev(ptr + v[k]);
                const int e = g.end(v[k]);
                const int ctx = g.vctx(v[k]);
                int p = p0 + 1, t = kNoTarget;
                for (; p < e; ++p) {
                    t = g.target(v[k], p, ctx);
                    if (ld_dev(dround + t) >= r) break;
                }
                if (p < e) {
                    edges += (uint64_t)(p - p0 + 1);
                    st_dev(ptr + v[k], p);
                    w[k] = t;
                    keep[k] = true;
                } else {
                    edges += (uint64_t)(e - p0);
                    st_dev(dround + v[k], r);
                }
            }
            int c = 0;
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) c += keep[k];
            int slot = block_append_base(c, cnt_out, nullptr, s_wave, &s_base);
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                if (keep[k]) {
                    st_dev(out + slot, v[k]);
                    st_dev(out + n + slot, w[k]);
                    ++slot;
                }
            }
        }
        if (!grid_barrier(ctr + kBarCount, ctr + kBarGen, ctr + kStall, budget)) break;
        if (ld_dev(cnt_out) == cnt_in) break;   // no removal in round r
    }
    edges = wave_sum(edges);
    if (lane_id() == 0 && edges) add_dev(worker_edges + blockIdx.x, edges);
    if (stats && blockIdx.x == 0 && threadIdx.x == 0) stats->rounds = (uint64_t)r;
}

// ------------------------------------------------------------ two-sided
// The constraint of Section 4.1 that also asks for a live predecessor: a second
// edge_index cursor runs over G^T.  In round r a vertex checks its successors
// first and, only if one is left, its predecessors; a vertex that finds no
// successor, or then no predecessor, is removed in round r.  Statuses are those
// of the round's start, so round r removes exactly the vertices of two-sided
// peeling step r, and the rounds number alpha + 1 of two-sided peeling.  A list
// entry carries both cursor targets, in three arrays of n ints.
struct List3 {
    int* v;    // vertex
    int* wo;   // successor at its out-cursor (kNoTarget: none)
    int* wi;   // predecessor at its in-cursor (kNoTarget: none)
};

__global__ void ac3_init2(ExplicitView out, ExplicitView in, int n, int* ptr, int* ptr_in,
                          int* dround, List3 l1, int* ctr, uint64_t* worker_edges, int P,
                          trim_stats_t* stats) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < kCtrInts) ctr[tid] = tid == kCnt0 + 1 ? n : 0;
    for (int p = tid; p < P; p += gridDim.x * blockDim.x) worker_edges[p] = 0;
    if (stats && tid < (int)(sizeof(trim_stats_t) / 8)) ((uint64_t*)stats)[tid] = 0;
    for (int v = tid; v < n; v += gridDim.x * blockDim.x) {
        const int b = out.begin(v), e = out.end(v), rb = in.begin(v), re = in.end(v);
        ptr[v] = b;
        ptr_in[v] = rb;
        dround[v] = INT_MAX;
        l1.v[v] = v;
        l1.wo[v] = b < e ? out.target(v, b, 0) : kNoTarget;
        l1.wi[v] = rb < re ? in.target(v, rb, 0) : kNoTarget;
    }
}

// The scan of one side after its cursor entry was found removed: from cursor
// position p0 + 1 on, the first entry not removed before round r.  Returns its
// position (the end if none) and the entry in t.
__device__ __forceinline__ int scan_on(const ExplicitView& g, int v, int p0, int e, int r,
                                       const int* dround, int& t) {
    int p = p0 + 1;
    t = kNoTarget;
    for (; p < e; ++p) {
        t = g.target(v, p, 0);
        if (ld_dev(dround + t) >= r) break;
    }
    return p;
}

__global__ __launch_bounds__(256) void ac3_rounds2(ExplicitView out, ExplicitView in, int n,
                                                   int* ptr, int* ptr_in, int* dround, List3 l0,
                                                   List3 l1, int* ctr, uint64_t* worker_edges,
                                                   trim_stats_t* stats, int budget) {
    __shared__ int s_wave[256 / kWave], s_base;
    uint64_t edges = 0;
    int r = 1;
    const int stride = gridDim.x * blockDim.x;
    for (;; ++r) {
        const List3 src = (r & 1) ? l1 : l0;
        const List3 dst = (r & 1) ? l0 : l1;
        const int cnt_in = ld_dev(ctr + kCnt0 + r % 3);
        int* cnt_out = ctr + kCnt0 + (r + 1) % 3;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st_dev(ctr + kCnt0 + (r + 2) % 3, 0);
            add_dev(ctr + kAcWork, cnt_in);
        }
        for (int base = blockIdx.x * blockDim.x; base < cnt_in; base += stride * kUnroll) {
            int v[kUnroll], wo[kUnroll], wi[kUnroll], dout[kUnroll], din[kUnroll];
            bool keep[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                const int i = base + k * stride + threadIdx.x;
                v[k] = -1;
                if (i < cnt_in) {
                    v[k] = ld_dev(src.v + i);
                    wo[k] = ld_dev(src.wo + i);
                    wi[k] = ld_dev(src.wi + i);
                }
            }
            // both cursor entries' removal rounds in flight together (the
            // predecessor's is only counted when a successor is left)
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                dout[k] = (v[k] >= 0 && wo[k] != kNoTarget) ? ld_dev(dround + wo[k]) : 0;
                din[k] = (v[k] >= 0 && wi[k] != kNoTarget) ? ld_dev(dround + wi[k]) : 0;
            }
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                keep[k] = false;
                if (v[k] < 0) continue;
                if (wo[k] != kNoTarget && dout[k] >= r) {   // successor cursor, checked again
                    edges += 1;
                } else {
                    const int p0 = ld_dev(ptr + v[k]), e = out.end(v[k]);
                    int t;
                    const int p = scan_on(out, v[k], p0, e, r, dround, t);
                    if (p >= e) {   // no successor left: removed in round r
                        edges += (uint64_t)(e - p0);
                        st_dev(dround + v[k], r);
                        continue;
                    }
                    edges += (uint64_t)(p - p0 + 1);
                    st_dev(ptr + v[k], p);
                    wo[k] = t;
                }
                if (wi[k] != kNoTarget && din[k] >= r) {   // predecessor cursor, checked again
                    edges += 1;
                    keep[k] = true;
                    continue;
                }
                const int p0 = ld_dev(ptr_in + v[k]), e = in.end(v[k]);
                int t;
                const int p = scan_on(in, v[k], p0, e, r, dround, t);
                if (p >= e) {   // no predecessor left: removed in round r
                    edges += (uint64_t)(e - p0);
                    st_dev(dround + v[k], r);
                    continue;
                }
                edges += (uint64_t)(p - p0 + 1);
                st_dev(ptr_in + v[k], p);
                wi[k] = t;
                keep[k] = true;
            }
            int c = 0;
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) c += keep[k];
            int slot = block_append_base(c, cnt_out, nullptr, s_wave, &s_base);
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                if (keep[k]) {
                    st_dev(dst.v + slot, v[k]);
                    st_dev(dst.wo + slot, wo[k]);
                    st_dev(dst.wi + slot, wi[k]);
                    ++slot;
                }
            }
        }
        if (!grid_barrier(ctr + kBarCount, ctr + kBarGen, ctr + kStall, budget)) break;
        if (ld_dev(cnt_out) == cnt_in) break;   // no removal in round r
    }
    edges = wave_sum(edges);
    if (lane_id() == 0 && edges) add_dev(worker_edges + blockIdx.x, edges);
    if (stats && blockIdx.x == 0 && threadIdx.x == 0) stats->rounds = (uint64_t)r;
}

struct Ac3Live {
    const int* dround;
    __device__ __forceinline__ bool operator()(int v) const { return dround[v] == INT_MAX; }
};

inline int grid_for(long long n, int block, int max_blocks = 1 << 20) {
    long long b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

template <class View>
hipError_t ac3_run(View g, int n, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                   uint64_t* worker_edges, trim_stats_t* stats, const uint32_t* preset = nullptr) {
    const int P = lc.workers;
    int pack_blocks = 0;
    // lists: 2n ints each (vertices, cursor targets) in the two 8n-byte arrays
    int* ptr = w.d;
    int* dround = w.c;
    int* list1 = reinterpret_cast<int*>(w.a);
    int* list0 = reinterpret_cast<int*>(w.b);
    {
        Timed t(lc, "ac3_init");
        hipLaunchKernelGGL(ac3_init<View>, dim3(grid_for(n, 256, 16384)), dim3(256), 0,
                           lc.stream, g, n, preset, ptr, dround, list1, w.ctr, worker_edges, P,
                           stats);
    }
    if (preset && n > 0) {
        Timed t(lc, "ac3_list_preset");
        hipLaunchKernelGGL(ac3_list_preset<View>, dim3(grid_for(n, 1024, lc.cus * 8)), dim3(256), 0,
                           lc.stream, g, n, preset, list1, w.ctr);
    }
    if (n > 0) {
        int nn = n;
        int budget = lc.budget;
        void* args[] = {&g,     &nn,          &ptr,          &dround, &list0,
                        &list1, (void*)&w.ctr, &worker_edges, &stats, &budget};
        {
            Timed t(lc, "ac3_rounds");
            hipError_t e = hipLaunchCooperativeKernel((const void*)ac3_rounds<View>, dim3(P),
                                                      dim3(256), args, 0, lc.stream);
            if (e != hipSuccess) return e;
        }
        Timed t(lc, "ac3_pack");
        pack_blocks = grid_for(n, 256, lc.cus * 4);
        hipLaunchKernelGGL(pack_bitmap<Ac3Live>, dim3(pack_blocks), dim3(256), 0, lc.stream,
                           Ac3Live{dround}, n, bitmap, w.part, w.ctr, nullptr, 0LL);
    }
    // an empty graph still runs the repeat-until loop once
    if (stats)
        hipLaunchKernelGGL(finalize_stats, dim3(1), dim3(1024), 0, lc.stream, n, P, 0, 0,
                           pack_blocks, 0, worker_edges, w.part, w.ctr, stats, 1);
    return hipGetLastError();
}

}  // namespace

// Two-sided rounds.  Working memory: cursors in w.d (successor side) and in
// the first n ints of x.rec_in (predecessor side), removal rounds in w.c; the
// two lists in w.a, w.b (vertex and successor entry) and x.hin (predecessor
// entry).  Two-sided AC-6 re-initialises x.hin and writes x.rec_in before
// reading it, so the calls can share them.
hipError_t ac3_two_csr(const trim_csr_t& g, const Work& w, const Work2& x, const LaunchCfg& lc,
                       uint32_t* bitmap, uint64_t* worker_edges, trim_stats_t* stats) {
    const int n = g.n, P = lc.workers;
    ExplicitView out{g.row_off, g.col}, in{g.rrow_off, g.rcol};
    int* ptr = w.d;
    int* ptr_in = reinterpret_cast<int*>(x.rec_in);
    int* dround = w.c;
    int* b = reinterpret_cast<int*>(w.b);
    List3 l1{w.a, w.a + n, x.hin};
    List3 l0{b, b + n, x.hin + n};
    int pack_blocks = 0;
    {
        Timed t(lc, "ac3t_init");
        hipLaunchKernelGGL(ac3_init2, dim3(grid_for(n, 256, 16384)), dim3(256), 0, lc.stream, out,
                           in, n, ptr, ptr_in, dround, l1, w.ctr, worker_edges, P, stats);
    }
    if (n > 0) {
        int nn = n;
        int budget = lc.budget;
        void* args[] = {&out, &in, &nn, &ptr, &ptr_in, &dround, &l0, &l1, (void*)&w.ctr,
                        &worker_edges, &stats, &budget};
        {
            Timed t(lc, "ac3t_rounds");
            hipError_t e = hipLaunchCooperativeKernel((const void*)ac3_rounds2, dim3(P), dim3(256),
                                                      args, 0, lc.stream);
            if (e != hipSuccess) return e;
        }
        Timed t(lc, "ac3t_pack");
        pack_blocks = grid_for(n, 256, lc.cus * 4);
        hipLaunchKernelGGL(pack_bitmap<Ac3Live>, dim3(pack_blocks), dim3(256), 0, lc.stream,
                           Ac3Live{dround}, n, bitmap, w.part, w.ctr, nullptr, 0LL);
    }
    if (stats)
        hipLaunchKernelGGL(finalize_stats, dim3(1), dim3(1024), 0, lc.stream, n, P, 0, 0,
                           pack_blocks, 0, worker_edges, w.part, w.ctr, stats, 1);
    return hipGetLastError();
}

hipError_t ac3_csr(const trim_csr_t& g, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                   uint64_t* worker_edges, trim_stats_t* stats, const uint32_t* preset) {
    ExplicitView v{g.row_off, g.col};
    return ac3_run(v, g.n, w, lc, bitmap, worker_edges, stats, preset);
}

hipError_t ac3_implicit(const trim_implicit_t& g, const Work& w, const LaunchCfg& lc,
                        uint32_t* bitmap, uint64_t* worker_edges, trim_stats_t* stats) {
    const int n = 1 << g.log2n;
    ImplicitView v{g.seed, g.zero_thr, g.deg_table, (uint32_t)(n - 1)};
    return ac3_run(v, n, w, lc, bitmap, worker_edges, stats);
}

int ac3_max_workers_per_cu(int) {
    int nb = 0, nb2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ac3_rounds<ExplicitView>, 256, 0) !=
        hipSuccess)
        return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, ac3_rounds<ImplicitView>, 256, 0) ==
            hipSuccess &&
        nb2 < nb)
        nb = nb2;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, ac3_rounds2, 256, 0) == hipSuccess &&
        nb2 < nb)
        nb = nb2;
    return nb < 1 ? 1 : nb;
}

}  // namespace trim
