// Launch interface between the host API (lattice_api.cpp) and the gfx950
// kernels (kernels.hip).  C++ linkage, library-internal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lat {

// Threshold table: index (nD+2)*1089 + (nV+16)*33 + (nJ+16).
constexpr int kTabD = 5, kTabV = 33, kTabJ = 33;
constexpr int kTabSize = kTabD * kTabV * kTabJ;  // 5445 uint32

// Scratch buffer layout (bytes).  Tracker (3 int64) and observable sums
// (7 int64) are adjacent so one 80-byte copy returns both.
constexpr size_t kScrTable = 0;
constexpr size_t kScrTrack = 22016;           // >= 4*kTabSize, 256-aligned
constexpr size_t kScrObs = kScrTrack + 3 * 8;  // 7 int64 follow the tracker
constexpr size_t kScrBytes = 24576;

// One phase of one sweep: phase p, displacement D = (r + 4m, 1 + 2k).
struct PhaseArgs {
    void *state;
    const uint32_t *thr;
    unsigned long long *track;  // 3 x int64 (two's complement) accumulators
    int L;
    int p, r, m, k;
    uint32_t key0, key1;
    uint32_t s_lo, s_hi;
};

hipError_t launch_phase_int8(const PhaseArgs &a, hipStream_t s);
hipError_t launch_phase_2bit(const PhaseArgs &a, hipStream_t s);
hipError_t launch_zero_i64(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_observables(const void *state, int L, int encoding, unsigned long long *obs, hipStream_t s);

}  // namespace lat
