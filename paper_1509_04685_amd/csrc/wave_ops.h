// Wave-level helpers shared by the kernels that count particles into bins (deposit sort,
// friends-of-friends cells).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cola {

// Wave-aggregated atomic increment by runs: consecutive lanes with equal keys share one atomic,
// and every run of the wave issues its atomic at once (one memory round trip per wave; particles
// in Lagrangian order give a few runs per wave).  Returns the old counter value plus the lane's
// rank in its run; equal keys in separate runs take separate slot ranges.
__device__ __forceinline__ uint32_t wave_increment(uint32_t* counter_base, uint32_t key, bool valid) {
    const int lane = __lane_id();
    const uint32_t prev_key = __shfl_up(key, 1);
    const int prev_valid = __shfl_up(valid ? 1 : 0, 1);
    const bool head = valid && (lane == 0 || prev_valid == 0 || prev_key != key);
    const unsigned long long hm = __ballot(head), vm = __ballot(valid);
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);  // lanes 0..lane
    uint32_t base = 0;
    if (head) {
        const unsigned long long brk = (hm | ~vm) & ~upto;  // where the runs after this lane start
        const int next = brk ? __ffsll((long long)brk) - 1 : 64;
        base = atomicAdd(&counter_base[key], (uint32_t)(next - lane));
    }
    const unsigned long long mine = hm & upto;
    const int my_head = mine ? 63 - __clzll((long long)mine) : lane;
    return __shfl(base, my_head) + (uint32_t)(lane - my_head);
}

}  // namespace cola
