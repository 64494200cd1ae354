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
};
enum SccMisc : int { kSccPivot = 0, kSccActive = 1, kSccChanged = 2, kSccTaken = 3,
                     kSccCount = 4, kSccEdges = 5, kSccMisc = 16 };

// Counts of one decomposition (host side).
struct SccCounts {
    long long n_scc = 0, trimmed = 0, giant = 0;
    int trims = 0, color_rounds = 0, color_sweeps = 0;
    long long search_edges = 0;   // list entries the searches examined
    double trim_ms = 0, search_ms = 0, color_ms = 0;   // host-timed phases
    bool stalled = false;   // a round made no progress (cannot happen; guarded)
};

// FW-BW decomposition driven from the host (synchronises `lc.stream`).
hipError_t scc_run(const trim_csr_t& g, const Work& w, const Work2& x, const SccWork& s,
                   const LaunchCfg& lc, int* label, SccCounts* counts);
int scc_max_workers_per_cu(int block);

}  // namespace trim
