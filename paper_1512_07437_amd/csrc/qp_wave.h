// Wavefront-level helpers shared by the gfx950 kernel sources.
#pragma once

#include <hip/hip_runtime.h>

#include "qp_internal.h"

namespace qp {

// inclusive prefix sum over the 64 lanes of a wavefront
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// counter[k] += 1 for every lane with `valid`, with one atomic per distinct k
// in the wavefront (the lanes of a wave mostly share a key, so per-lane
// atomics on a few addresses would serialise); returns the lane's 0-based
// position among all additions to counter[k].  Uniform control flow: every
// lane of the wave must call it.
__device__ __forceinline__ int wave_count_add(int* counter, int k, bool valid) {
    const int lane = threadIdx.x & (kWave - 1);
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    unsigned long long todo = __ballot(valid);
    int slot = 0;
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const int lk = __shfl(k, leader, kWave);
        const bool mine = valid && k == lk;
        const unsigned long long same = __ballot(mine);
        int base = 0;
        if (lane == leader) base = atomicAdd(&counter[lk], __popcll(same));
        base = __shfl(base, leader, kWave);
        if (mine) slot = base + __popcll(same & below);
        todo &= ~same;
    }
    return slot;
}

}  // namespace qp
