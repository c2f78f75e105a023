// ra_tune.hpp — tile selection: beads per lane M for each group.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "ra.h"

namespace ra {

// Beads-per-lane values compiled into each kernel family.
const std::vector<int>& family_beads_per_lane(int family);

// Cost model: a wavefront of P = floor(64 / ceil(N/M)) replicas costs M lane
// slots per bead-step, so a group costs M * ceil(R/P); the cheapest legal M
// wins, ties going to the smaller M (more wavefronts in flight). `forced`
// (> 0) is used when it is legal for N and the noise map. Noise map 2 takes
// only multiples of four (map_allows).
bool map_allows(int nmap, int M);
int choose_beads_per_lane(int n_beads, int n_replicas, int family, int forced, int nmap);

// Times every legal M for each distinct (N, spring) of the batch with a short
// run of the fused kernel that fills every SIMD four times and keeps the
// fastest per replica. With waves_per_block = 0 on entry it also tries 1, 2
// and 4 wavefronts per workgroup and returns the size whose tiles give the
// least predicted batch time (sum over groups of R x time per replica).
// Results are kept per process and, if RA_AUTOTUNE_CACHE names a file, in that
// JSON-lines file (read when a context first uses it).
ra_status autotune_tiles(const std::vector<ra_chain_desc>& descs, const ra_run_desc& run, int family,
                         int& waves_per_block, hipStream_t stream, std::vector<int>& Ms, std::string& why);

}  // namespace ra
