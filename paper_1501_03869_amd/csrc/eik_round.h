// The end of one relaxation round of the travel-time tables (Section II-B):
// the counters a round's workgroups update, and how the host learns the next
// round's size without a copy command or a stream synchronisation.
//
// counters (device, EIK_COUNTERS words, zeroed once before the first round):
//   [0] tiles appended to the next round's list
//   [1] unused, 0
//   [2..3] relaxation sweeps so far (64-bit)
// host (pinned, EIK_HOST_WORDS words):
//   [0..3] copied from counters[0..3] after each round
//   [4] the sequence number of the last round copied
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <chrono>

namespace pat_eik {

constexpr int EIK_COUNTERS = 4;
constexpr int EIK_HOST_WORDS = 8;

namespace {

// One thread, launched after a round's tile kernel on the same stream, so
// that every counter update of the round has landed: copies the counters to
// the host words, then (after a system-scope fence) the round's sequence
// number, and clears the next-round count.
__global__ void __launch_bounds__(64) k_eik_round_end(uint32_t *__restrict__ counters, uint32_t *host, uint32_t seq) {
    if (threadIdx.x != 0) return;
    host[0] = counters[0];
    host[1] = counters[1];
    host[2] = counters[2];
    host[3] = counters[3];
    __threadfence_system();
    *(volatile uint32_t *)&host[4] = seq;
    counters[0] = 0u;
}

// Waits on the host until round seq's words are in: it polls the sequence
// word for up to spin_ms (0: not at all), then falls back to synchronising
// the stream, after which the words are final either way.  The GPU never
// waits on the host.
static inline hipError_t wait_round(volatile const uint32_t *host, uint32_t seq, hipStream_t st,
                                    double spin_ms) {
    if (spin_ms <= 0.0) return hipStreamSynchronize(st);
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned it = 1;; ++it) {
        if (host[4] == seq) return hipSuccess;
        if ((it & 1023u) == 0 &&
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() > spin_ms)
            return hipStreamSynchronize(st);
    }
}

}  // namespace

}  // namespace pat_eik
