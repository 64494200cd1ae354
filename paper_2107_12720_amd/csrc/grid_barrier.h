// grid_barrier.h -- a grid-wide barrier for kernels whose workgroups are all
// resident at once (the AC-3 rounds, launched cooperatively, and the AC-6
// forest-collapse rounds, at most two workgroups per CU), with a watchdog.
#pragma once
#include "trim_device.h"

namespace trim {

// Sense-free grid barrier: arrivals counted in *count, the last arrival resets
// it and bumps *gen.  Everything a round shares with later rounds (lists,
// cursors, removal rounds) is written and read with device-coherent accesses,
// so arriving after one's own stores have completed (s_waitcnt) is enough; no
// agent-scope fence (a whole-L2 write-back and invalidate on gfx950) runs.
// The generation must be read before arriving: the two accesses go to
// different addresses, and without the wait in between the read can be
// performed after the last arrival has already bumped *gen; the block would
// then wait for a release that never comes.
// Watchdog: a workgroup that has polled `budget` times without a release, or
// that finds the stall word raised, gives up and raises it.  Returns false
// (the same in every thread of the block) when the rounds must be abandoned.
__device__ __forceinline__ bool grid_barrier(int* count, int* gen, int* stall, int budget) {
    __shared__ int s_go;
    complete_mem();
    __syncthreads();
    if (threadIdx.x == 0) {
        int go = 1;
        const int g0 = ld_dev(gen);
        complete_mem();   // g0 is read before this block can complete the barrier
        if (add_dev(count, 1) == (int)gridDim.x - 1) {
            st_dev(count, 0);
            complete_mem();
            add_dev(gen, 1);
        } else {
            for (int polls = 1; ld_dev(gen) == g0; ++polls) {
                if (polls > budget || ((polls & 63) == 0 && ld_dev(stall))) {
                    st_dev(stall, 1);
                    go = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        s_go = go && ld_dev(stall) == 0;
    }
    __syncthreads();
    const bool go = s_go != 0;
    __syncthreads();   // s_go is rewritten by the next barrier
    return go;
}

}  // namespace trim
