// The end of one relaxation round of the travel-time tables (Section II-B):
// the counters a round's workgroups update, and how the host learns the next
// round's size with one stream synchronisation and no copy command.
//
// counters (device, EIK_COUNTERS words, zeroed once before the first round):
//   [0] tiles appended to the next round's list
//   [1] unused, 0
//   [2..3] relaxation sweeps so far (64-bit)
// host (pinned, 4 words): [0..3] copied from counters[0..3] after each round.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pat_eik {

constexpr int EIK_COUNTERS = 4;

namespace {

// One thread, launched after a round's tile kernel on the same stream, so
// that every counter update of the round has landed: copies the counters to
// the host words and clears the next-round count.
__global__ void __launch_bounds__(64) k_eik_round_end(uint32_t *__restrict__ counters, uint32_t *__restrict__ host) {
    if (threadIdx.x != 0) return;
    host[0] = counters[0];
    host[1] = counters[1];
    host[2] = counters[2];
    host[3] = counters[3];
    __threadfence_system();
    counters[0] = 0u;
}

}  // namespace

}  // namespace pat_eik
