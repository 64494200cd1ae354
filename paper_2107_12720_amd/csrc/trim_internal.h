// trim_internal.h -- host-side declarations shared by the kernel files and the
// C-ABI layer of libtrim.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/trim.h"

namespace trim {

// Counter slots of the per-call control block (int32 unless noted).
// Hot words sit 128 bytes apart so that they live in different cache lines
// (and L2 channels): pollers of one do not queue behind atomics on another.
enum Ctr : int {
    kQHead = 0,      // next queue slot to hand out
    kQTail = 32,     // slots reserved by producers
    kPending = 64,   // queued items + workers holding private work
    kBad = 96,       // validation failures
    kBarCount = 128, // grid barrier arrivals
    kBarGen = 160,   // grid barrier generation
    kCursor = 192,   // next unclaimed vertex of the chunked sweep
    kJCnt0 = 200,    // AC-6 forest collapse: list sizes, rotating over 3 slots
    kJDone0 = 204,   // vertices whose root was found, per round, rotating over 3 slots
    kJStop = 208,    // nonzero once the pointer-jumping rounds are over
    kJRounds = 209,  // rounds run
    kJKilled = 210,  // vertices removed by the collapse
    kJWork = 211,    // list entries the collapse rounds processed
    kLvCnt0 = 212,   // AC-6 level-synchronous phases: list sizes, rotating over 3 slots
    kLvPhases = 215, // phases run
    kAcWork = 216,   // AC-3: live-list entries processed over all rounds
    kCnt0 = 224,     // AC-3 live-list sizes, rotating over 3 slots
    kStall = 240,    // watchdog: nonzero once a persistent kernel gave up (opts.budget)
    // AC-6 with late support registration (opts.rounds): the round list's
    // size, removals per round (rotating over 3 slots), the stop word (set
    // once a round removed nothing), the rounds run and the cursor re-checks
    kHyCnt0 = 4,
    kHyDead0 = 36,
    kHyStop = 100,
    kHyRounds = 101,
    kHyWork = 102,   // uint64 (words 102 and 103, 8-byte aligned)
    kCtrInts = 256
};

static_assert(kHyWork % 2 == 0, "the 64-bit re-check counter needs an 8-byte aligned word");

// Working memory of one call, sized for n vertices (owned by trim_ctx).
struct Work {
    int* a = nullptr;         // 2n int32: AC-6 (out-side) list heads / AC-4 counters /
                              //   AC-3 list
    uint64_t* b = nullptr;    // n uint64: AC-6 (out-side) records / AC-3 list
    int* c = nullptr;         // n int32: AC-6 bitmap of vertices removed at the start /
                              //   AC-3 removal round
    int* d = nullptr;         // n int32: AC-3 cursor / two-sided AC-4 removal flags /
                              //   batch: first vertex of each vertex's graph (union
                              //   path) or the graphs' claim order (owned path)
    uint32_t* e = nullptr;    // 2n uint32: AC-6 forest-collapse lists / phase lists (two of n)
    int* jp = nullptr;        // n int32: AC-6 forest links
    int* ext = nullptr;       // (kMoreLists - 1) n int32: the split S_more heads of AC-6
                              //   (allocated only for capacities up to kSplitMaxN)
    uint32_t* q = nullptr;    // 3n shared-queue slots ((2 + kMoreLists) n with ext), kNone
                              //   between calls
    long long qwords = 0;     // size of q in words (slack included)
    int* ctr = nullptr;       // kCtrInts control words
    uint64_t* wedges = nullptr;  // per-worker counts when the caller has none (batches)
    uint64_t* part = nullptr;    // per-block partial sums (kPartSlots x kPartStride)
    long long cap = 0;           // vertices the per-vertex buffers hold
    int* hl = nullptr;           // AC-6 with late support registration: the round list,
                                 //   2 * hcap ints (vertex, cursor target and flags), then
                                 //   3 round filters of up to 2^kRoundFilterMaxLog2 bits
    long long hcap = 0;
};
// Extra working memory of two-sided AC-6 (allocated on its first use).
struct Work2 {
    int* hin = nullptr;         // 2n int32: in-side list heads
    uint64_t* rec_in = nullptr; // n uint64: in-side (next, cursor) records
    uint32_t* q = nullptr;      // kQueuePerVertexTwo(Split) n shared-queue slots (+ kQueueSlots),
                                //   kNone between calls
    long long qwords = 0;       // size of q in words
};
constexpr int kMaxWorkers = 16384;
// Round filters of late support registration: at most 2^18 bits (32 KB) each,
// so that a round workgroup can hold one in LDS.
constexpr int kRoundFilterMaxLog2 = 18;
// AC-6 splits S_more lists kMoreLists ways for graphs up to kSplitMaxN
// vertices; a close can then queue up to kMoreLists S_more heads, so the
// shared queue needs room for 2 + kMoreLists items per vertex instead of 3.
constexpr int kMoreListsLog = 2;
constexpr int kMoreLists = 1 << kMoreListsLog;
constexpr long long kSplitMaxN = 1LL << 25;
constexpr int kQueuePerVertexSplit = 2 + kMoreLists;
// Two-sided AC-6 queues at most 7 items per vertex with one S_more list per
// side (one close, one S_last member per side, one S_more list head per side,
// one failed scan per side), kMoreLists - 1 more with split out-side lists;
// one slot per vertex more is kept as a margin.
constexpr int kQueuePerVertexTwo = 8;
constexpr int kQueuePerVertexTwoSplit = kQueuePerVertexTwo + kMoreLists - 1;
// shared-queue slack beyond 3n slots: outstanding tickets, 64 per wavefront
constexpr int kQueueSlots = 64 * 4 * kMaxWorkers;
constexpr int kPartStride = 16384;   // >= workers, sweep blocks and pack blocks
enum PartSlot : int { kPartCloses = 0, kPartJoins = 1, kPartVisited = 2, kPartSweep = 3,
                      kPartLive = 4, kPartDeg = 5, kPartQhw = 6, kPartLiveEdges = 7,
                      kPartLvCloses = 8, kPartLvJoins = 9, kPartLvVisited = 10,
                      kPartSlots = 11 };

// Optional per-kernel event timing (trim_ctx_set_timing): event pairs of up to
// kMax kernels per call, for each of the last `keep` calls (a ring of kCalls
// slots), so that a timed loop need not wait for every call.
struct Timer {
    static constexpr int kMax = 16;
    static constexpr int kCalls = 64;
    struct Slot {
        hipEvent_t ev[2 * kMax] = {};
        const char* names[kMax] = {};
        int count = 0;
    };
    Slot slot[kCalls];
    int keep = 0;          // slots in use (0: timing off)
    long long calls = 0;   // calls recorded since timing was set
    int created = 0;       // slots whose events exist
    // The slot for a new call; its previous contents are dropped.
    Slot* next() {
        Slot* s = &slot[calls++ % keep];
        s->count = 0;
        return s;
    }
};

struct LaunchCfg;
// Records events around the kernels launched while it is alive.
class Timed {
  public:
    Timed(const LaunchCfg& lc, const char* name);
    ~Timed();

  private:
    Timer::Slot* t_;
    hipStream_t s_;
    int idx_ = -1;
};

struct LaunchCfg {
    int block = 256;          // sweep block size
    int chunk = 0;            // vertices per dynamically claimed sweep chunk (0 = automatic)
    int schedule = 0;         // TRIM_SCHED_* perturbation flags (tests)
    int workers = 0;          // persistent workgroups
    int budget = TRIM_DEFAULT_BUDGET;   // watchdog step budget (opts.budget)
    bool forest = true;       // AC-6: collapse the last-successor forest after the sweep
    int rounds = 0;           // AC-6: rounds before supports are registered (opts.rounds)
    int cus = 256;
    hipStream_t stream = nullptr;
    Timer::Slot* timer = nullptr;   // non-null: record per-kernel events here
};

// Vertices per dynamically claimed chunk of a first sweep: opts.chunk when
// given, else 4096 (the paper's s, Section 8) cut down for small graphs so
// that there are at least four chunks per CU, but never below 256; rounded up
// to a multiple of the block size.
inline int sweep_chunk(const LaunchCfg& lc, long long n, int block) {
    long long c = lc.chunk;
    if (c <= 0) {
        c = n / (4LL * (lc.cus > 0 ? lc.cus : 1));
        c = c < 256 ? 256 : (c > 4096 ? 4096 : c);
    }
    return (int)((c + block - 1) / block * block);
}

inline Timed::Timed(const LaunchCfg& lc, const char* name) : t_(lc.timer), s_(lc.stream) {
    if (t_ && t_->count < Timer::kMax) {
        idx_ = t_->count++;
        t_->names[idx_] = name;
        (void)hipEventRecord(t_->ev[2 * idx_], s_);
    }
}
inline Timed::~Timed() {
    if (idx_ >= 0) (void)hipEventRecord(t_->ev[2 * idx_ + 1], s_);
}

// ------------------------------------------------------------------ AC-6
// preset: optional device bitmap of vertices removed before trimming (NULL = none)
hipError_t ac6_csr(const trim_csr_t& g, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                   uint64_t* worker_edges, trim_stats_t* stats, const uint32_t* preset = nullptr);
hipError_t ac6_implicit(const trim_implicit_t& g, const Work& w, const LaunchCfg& lc,
                        uint32_t* bitmap, uint64_t* worker_edges, trim_stats_t* stats);
// trim_batch with one workgroup per graph (batch.hip); the default.
hipError_t ac6_batch_owned(int G, const int64_t* vbase, const int32_t* row_off,
                           const int32_t* col, int64_t total_n, const int64_t* bitmap_base,
                           const Work& w, const LaunchCfg& lc, uint32_t* bitmaps,
                           uint64_t* graph_edges, trim_stats_t* stats);
int ac6_owned_blocks_per_cu(int block);
hipError_t ac6_batch(int G, const int64_t* vbase, const int32_t* row_off, const int32_t* col,
                     int64_t total_n, const int64_t* bitmap_base, const Work& w,
                     const LaunchCfg& lc, uint32_t* bitmaps, uint64_t* graph_edges,
                     trim_stats_t* stats);
int ac6_max_workers_per_cu(int block);
hipError_t ac6_two_csr(const trim_csr_t& g, const Work& w, const Work2& x, const LaunchCfg& lc,
                       uint32_t* bitmap, uint64_t* worker_edges, trim_stats_t* stats);
int ac6_two_max_workers_per_cu(int block);

// ------------------------------------------------------------------ AC-4
hipError_t ac4_csr(const trim_csr_t& g, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                   uint64_t* worker_edges, trim_stats_t* stats, const uint32_t* preset = nullptr);
hipError_t ac4_two_csr(const trim_csr_t& g, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                       uint64_t* worker_edges, trim_stats_t* stats);
int ac4_max_workers_per_cu(int block);

// ------------------------------------------------------------------ AC-3
hipError_t ac3_csr(const trim_csr_t& g, const Work& w, const LaunchCfg& lc, uint32_t* bitmap,
                   uint64_t* worker_edges, trim_stats_t* stats, const uint32_t* preset = nullptr);
hipError_t ac3_implicit(const trim_implicit_t& g, const Work& w, const LaunchCfg& lc,
                        uint32_t* bitmap, uint64_t* worker_edges, trim_stats_t* stats);
hipError_t ac3_two_csr(const trim_csr_t& g, const Work& w, const Work2& x, const LaunchCfg& lc,
                       uint32_t* bitmap, uint64_t* worker_edges, trim_stats_t* stats);
int ac3_max_workers_per_cu(int block);

// ------------------------------------------------------------ learned order
// Edge-parallel tiles of the preprocessing and reordering kernels: the
// scratch they need is tile_scratch_ints(m) ints.
constexpr int kTileE = 4096;
inline long long tile_scratch_ints(long long m) {
    const long long T = (m + kTileE - 1) / kTileE;
    const long long B = (T + 1 + 63) / 64;   // chunks of 64 scan rows
    return 3 * T + (T + 1) * 16 + B * 16;
}
// Per-XCD in-degree copies (kXcdCopies * n ints) are used up to this n.
constexpr int kXcdCopies = 8;
constexpr int kXcdCopiesMaxN = 1 << 26;
hipError_t mlp_prepare(const int* row_off, const int* col, int n, long long m, int* indeg,
                       int* src, int* tinfo, int* copies, hipStream_t s);
hipError_t mlp_grad_launch(const int* row_off, const int* col, const int* indeg, const int* src,
                           long long m, const uint32_t* live, const short* pbf,
                           const long long* ids, long long count, uint64_t seed, int step,
                           float* grad, int cus, hipStream_t s);
hipError_t mlp_adam_launch(float* p32, short* pbf, float* m1, float* m2, float* grad, float lr,
                           float beta1, float beta2, float eps, int step, hipStream_t s);
hipError_t mlp_score_launch(const int* row_off, const int* col, const int* indeg, const int* src,
                            int n, long long m, const short* pbf, float* score, float2* vf,
                            int cus, hipStream_t s);
hipError_t edge_keys_launch(const int* row_off, const int* col, long long m, int kind,
                            uint64_t seed, float* key, hipStream_t s);
hipError_t order_launch(const int* row_off, const int* col, int n, long long m, const float* key,
                        float lo, float hi, int* col_out, int* tinfo, int* tcnt,
                        hipStream_t s);

// ------------------------------------------------------------ validation
hipError_t validate_csr(const trim_csr_t& g, const Work& w, hipStream_t s);
// The calling thread's error message (trim_last_error) and the option checks
// of trim_api.hip, for entry points defined in other files.
int report_error(int code, const char* msg);
int check_options(const trim_opts_t* o);

}  // namespace trim
