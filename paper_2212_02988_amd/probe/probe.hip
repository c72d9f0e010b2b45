// Gather-rate probe (measurement aid, built into its own library and not
// part of the C ABI of include/prism.h): the rate at which the CUs issue
// 64-lane 4-byte loads from a buffer small enough to stay in the caches,
// with the lanes of a load reading consecutive words (one or two cache
// lines per load) or independent random words (up to 64 lines per load).
// The benchmark places the renderer's measured vector-load rate between
// these two ceilings: its map reads are gathers from an L2- and L1-resident
// footprint, so neither HBM bandwidth nor a streaming copy bounds them.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// Each lane issues 8 independent loads per round, `rounds` rounds.  random:
// word index from the top bits of a per-lane linear congruential sequence
// (shift = 32 - log2(words)); else the lanes of a wave read consecutive
// words, each load of a round a different run of 64.  The loads feed a sum
// that is stored only if it takes a value the data cannot give (the buffer
// holds non-negative numbers), which keeps every load live.
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ buf, uint32_t words_mask, int shift,
                                                int rounds, int random, float* __restrict__ sink) {
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    uint32_t s = gid * 2654435761u + 12345u;
    float acc = 0.0f;
    for (int it = 0; it < rounds; ++it) {
        uint32_t idx[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (random) {
                s = s * 1664525u + 1013904223u;
                idx[j] = s >> shift;
            } else {
                idx[j] = (gid + (uint32_t)(it * 8 + j) * 64u * 131u) & words_mask;
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += buf[idx[j]];
    }
    if (acc < 0.0f) sink[0] = acc;
}

}  // namespace

// buf: device float [words], words a power of two in [64, 2^30], all values
// >= 0; sink: device float [1] (written only if the sum were negative).
// blocks workgroups of 256 threads, each lane 8 * rounds loads.  Returns a
// hipError_t (hipErrorInvalidValue for bad arguments; nothing launched).
extern "C" int prism_probe_gather(const float* buf, uint64_t words, int rounds, int random, int blocks, float* sink,
                                  hipStream_t stream) {
    if (!buf || !sink || words < 64 || words > (1ull << 30) || (words & (words - 1)) || rounds < 1 || blocks < 1)
        return (int)hipErrorInvalidValue;
    int log2w = 0;
    while ((1ull << log2w) < words) ++log2w;
    k_gather<<<blocks, 256, 0, stream>>>(buf, (uint32_t)(words - 1), 32 - log2w, rounds, random, sink);
    return (int)hipGetLastError();
}
