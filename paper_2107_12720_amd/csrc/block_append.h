// block_append.h -- appending to a shared list from a whole workgroup with one
// counter update: a counter that every wavefront bumps on its own becomes a
// single-address hot spot (about 65,000 serialised atomics per 2^22 items).
#pragma once
#include "trim_device.h"

namespace trim {

// Every thread of the block offers `cnt` items (cnt <= K); returns the slot of
// this thread's first item.  One fetch-add on *tail (and on *pending, if
// given) per call.  All threads of the block must call it; it synchronises.
// s_wave holds one int per wavefront, s_base one int.
__device__ __forceinline__ int block_append_base(int cnt, int* tail, int* pending, int* s_wave,
                                                 int* s_base) {
    int inc = cnt;
    for (int d = 1; d < kWave; d <<= 1) {
        const int t = __shfl_up(inc, d);
        if (lane_id() >= d) inc += t;
    }
    const int wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    if (lane_id() == kWave - 1) s_wave[wv] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int total = 0;
        for (int w = 0; w < nw; ++w) {
            const int x = s_wave[w];
            s_wave[w] = total;
            total += x;
        }
        int base = 0;
        if (total) {
            if (pending) add_dev(pending, total);
            base = add_dev(tail, total);
        }
        *s_base = base;
    }
    __syncthreads();
    const int slot = *s_base + s_wave[wv] + inc - cnt;
    __syncthreads();   // s_wave / s_base may be reused by the next call
    return slot;
}

}  // namespace trim
