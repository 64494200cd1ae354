// scc_internal.h -- host-side declarations of the SCC decomposition and of the
// preset form of two-sided AC-6 it drives.  Not part of the public interface.
#pragma once
#include "trim_internal.h"

namespace trim {

// Two-sided AC-6 with the vertices of `preset` (device bitmap, may be NULL)
// removed before it starts.
hipError_t ac6_two_csr_preset(const trim_csr_t& g, const Work& w, const Work2& x,
                              const LaunchCfg& lc, uint32_t* bitmap, uint64_t* worker_edges,
                              trim_stats_t* stats, const uint32_t* preset);

// Working memory of trim_scc, sized for n vertices.
struct SccWork {
    uint32_t* assigned = nullptr;  // ceil(n/32) + 64 words: vertices whose component is known
    uint32_t* live = nullptr;      // ceil(n/32) + 64 words: survivors of the last trim
    int* flags = nullptr;          // n: reach marks, bit 0 forward, bit 1 backward
    int* color = nullptr;          // n: max-label colours
    unsigned long long* misc = nullptr;  // kSccMisc words: pivot key, counters
    uint32_t* front[2] = {nullptr, nullptr};  // 2n + 64 search items each (current, next)
    uint32_t* pre = nullptr;       // 2n + 64: exclusive prefix of the frontier's list lengths
    uint32_t* bsum = nullptr;      // per-chunk sums of the prefix scan
};
enum SccMisc : int { kSccPivot = 0, kSccActive = 1, kSccChanged = 2, kSccTaken = 3,
                     kSccCount = 4, kSccEdges = 5, kSccFront = 6, kSccTotal = 7, kSccNext = 8,
                     kSccLevels = 9, kSccOrs = 10, kSccMisc = 16 };
constexpr int kScanChunk = 1024;   // frontier items per chunk of the prefix scan

// Counts of one decomposition (host side).
struct SccCounts {
    long long n_scc = 0, trimmed = 0, giant = 0;
    int trims = 0, color_rounds = 0, color_sweeps = 0;
    long long search_edges = 0;   // list entries the searches examined
    int search_levels = 0;        // frontier levels of all searches
    long long search_ors = 0;     // mark fetch-ors issued (marks won: at most 2 per vertex)
    long long paired = 0;         // vertices found in components of two by the size-2 check
    double size2_ms = 0;
    double trim_ms = 0, search_ms = 0, color_ms = 0;   // host-timed phases
    bool stalled = false;   // a round made no progress (cannot happen; guarded)
};

// Size-2 check on the vertices not in `preset` (NULL = all): partner[u] (n
// ints) as in trim_size2; n_paired (host, may be NULL: then no
// synchronisation) receives the number of paired vertices.  Uses s.live,
// s.flags, s.color and s.misc.
hipError_t size2_run(const trim_csr_t& g, const SccWork& s, const uint32_t* preset, int* partner,
                     long long* n_paired, hipStream_t st, int cus);

// FW-BW decomposition driven from the host (synchronises `lc.stream`).
hipError_t scc_run(const trim_csr_t& g, const Work& w, const Work2& x, const SccWork& s,
                   const LaunchCfg& lc, int* label, SccCounts* counts);

}  // namespace trim
