// Launch interface between the host API (lattice_api.cpp) and the gfx950
// kernels (kernels.hip).  C++ linkage, library-internal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lat {

// Threshold table of the method, over nD in [-2,2], nV, nJ in [-16,16]:
// index (nD+2)*1089 + (nV+16)*33 + (nJ+16).
constexpr int kTabV = 33, kTabJ = 33;
constexpr int kTabSize = 5 * kTabV * kTabJ;  // 5445

// Device form of the threshold table.  A pair move changes the charged count
// by 0 or +-2, so only the slices nD in {-2, 0, 2} are reachable; entry
// (nD/2+1)*1089 + (nV+16)*33 + (nJ+16) holds {threshold, packed triple}
// where packed = 1<<27 | (nD+2)<<20 | (nV+16)<<10 | (nJ+16) is what an
// accepted move adds to the per-thread energy tracker.
constexpr int kDevTabEntries = 3 * kTabV * kTabJ;  // 3267 x uint2
// Transition table: entry st*6 + j for pair state st = code_a | code_b<<2 and
// choice j: {coef, meta}.  coef = int8x4 (33*dS_a, 33*dS_b, dsig_a, dsig_b);
// meta = C | new_state<<16, with C chosen so that
// dot4(coef, (sumS_a+4, sumS_b+4, sumsig_a+4, sumsig_b+4)) + C is the
// device-table index of the move's (nD, nV, nJ).
constexpr int kTransEntries = 16 * 6;

// Scratch buffer layout (bytes).  Tracker (3 int64) and observable sums
// (7 int64) are adjacent so one 80-byte copy returns both.
constexpr size_t kScrDevTab = 0;                      // 3267 x 8 = 26136
constexpr size_t kScrTrans = 26368;                   // 96 x 8 = 768
constexpr size_t kScrTrack = 27136;                   // 3 x int64
constexpr size_t kScrObs = kScrTrack + 3 * 8;         // 7 x int64
constexpr size_t kScrBytes = 32768;

// One phase of one sweep: phase p, displacement D = (r + 4m, 1 + 2k).
struct PhaseArgs {
    void *state;
    const uint2 *dev_tab;    // kDevTabEntries
    const uint2 *trans;      // kTransEntries
    unsigned long long *track;  // 3 x int64 (two's complement) accumulators
    int L;
    int p, r, m, k;
    uint32_t key0, key1;
    uint32_t s_lo, s_hi;
};

// Launch shape of the 2-bit phase kernel: rows of the a-class per block
// (0 = automatic) and blocks per compute unit.
struct Tuning2Bit {
    int rows_per_block;
    int blocks_per_cu;
};

hipError_t launch_phase_int8(const PhaseArgs &a, hipStream_t s);
hipError_t launch_phase_2bit(const PhaseArgs &a, const Tuning2Bit &t, hipStream_t s);
hipError_t launch_zero_i64(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_observables(const void *state, int L, int encoding, unsigned long long *obs, hipStream_t s);

}  // namespace lat
