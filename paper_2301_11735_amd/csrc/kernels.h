// Launch interface between the host API (lattice_api.cpp) and the gfx950
// kernels (phase.hip, obs.hip, batch.hip).  C++ linkage, library-internal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lat {

// Threshold table of the method, over nD in [-2,2], nV, nJ in [-16,16]:
// index (nD+2)*1089 + (nV+16)*33 + (nJ+16).
constexpr int kTabV = 33, kTabJ = 33;
constexpr int kTabSize = 5 * kTabV * kTabJ;  // 5445

// Device form of the threshold table, compacted to the triples a pair move
// can reach: a move that changes the charged count (nD = +-2) or a q = +-1
// move has |nV|, |nJ| <= 8; a charge swap (+,-) <-> (-,+) has nD = nJ = 0 and
// |nV| <= 16; a spin change of both-spin or one-spin pairs has nD = nV = 0
// and |nJ| <= 16.  Regions (entries {threshold, packed triple}):
//   slice s = nD/2 + 1:  289*s + (nV+8)*17 + (nJ+8)     |nV|, |nJ| <= 8
//   V line (nD = nJ = 0): kDevVLine + nV + 16
//   J line (nD = nV = 0): kDevJLine + nJ + 16
// packed = 1<<27 | (nD+2)<<20 | (nV+16)<<10 | (nJ+16) is what an accepted
// move adds to the per-thread energy tracker.
constexpr int kDevSlice = 17 * 17;
constexpr int kDevVLine = 3 * kDevSlice;       // 867
constexpr int kDevJLine = kDevVLine + 33;      // 900
constexpr int kDevTabEntries = kDevJLine + 33; // 933 x uint2
// Transition table: entry st*6 + j for pair state st = code_a | code_b<<2 and
// choice j: {coef, meta}.  coef = int8x4 applied to the packed neighbour sums
// (sumS_a+4, sumS_b+4, sumsig_a+4, sumsig_b+4); meta = C | new_state<<16, with
// C chosen so that dot4(coef, sums) + C is the move's device-table index.
constexpr int kTransEntries = 16 * 6;

// Scratch buffer layout (bytes).  The tracker total (3 int64), observable
// sums (7 int64) and error flags are adjacent so one 88-byte copy returns all.
// Partial sums are gathered without contended atomics: the phase kernels add
// block b's tracker sums into tracker slot b, the observable reduction writes
// block b's sums into observable slot b, single-block kernels add into the
// tracker base; k_fold_sums folds slots into the totals.
constexpr size_t kScrDevTab = 0;                      // 933 x 8 = 7464
constexpr size_t kScrTrans = 7680;                    // 96 x 8 = 768
constexpr size_t kScrTrack = 8448;                    // 3 x int64: tracker total (output)
constexpr size_t kScrObs = kScrTrack + 3 * 8;         // 7 x int64: observable sums (output)
constexpr size_t kScrErr = kScrObs + 7 * 8;           // uint32 error flags (bit 0: barrier time-out)
constexpr size_t kScrBarrier = 8576;                  // uint32 phase-barrier counter (+ 4 spare bytes)
constexpr size_t kScrDesc = 8704;                     // LatDesc
constexpr size_t kScrTrackBase = 8768;                // 3 x int64 from single-block kernels
constexpr size_t kScrObsSlots = 9216;                 // kMaxObsSlots x 7 x int64
constexpr int kMaxObsSlots = 256;
constexpr size_t kScrSlots = 24576;                   // kMaxSlots x 3 x int64 from the phase kernels
constexpr int kMaxSlots = 1024;
constexpr size_t kScrFullTab = kScrSlots + (size_t)kMaxSlots * 24;  // 49152: kTabSize x uint32 thresholds
// Penalty mode: thresholds over (nD, nV, nJ, dS) of one site, nD in [-1, 1],
// nV and nJ in [-8, 8], dS in [-2, 2], index ((nD+1)*17 + nV+8)*17 + nJ+8)*5 + dS+2.
constexpr int kMuTabSize = 3 * 17 * 17 * 5;  // 4335
constexpr size_t kScrMuTab = kScrFullTab + ((size_t)kTabSize * 4 + 255) / 256 * 256;  // 71168
// Delta form of the transition table, read by the 2-bit phase kernel: entry
// st*6 + j is {coef, C, R, 0} with coef and C as in the transition table and
// R = (d_a * 0x5555) | (d_b * 0x5555) << 16, where d_a and d_b are the XOR of
// the new and the old code of site a and of site b: every 2-bit field of the
// low half holds d_a and every field of the high half d_b, so that one AND
// with a field mask places an accepted move's code changes at any pair
// position.
constexpr size_t kScrTransD = kScrMuTab + ((size_t)kMuTabSize * 4 + 255) / 256 * 256;  // 88576
constexpr size_t kScrBytes = kScrTransD + (size_t)kTransEntries * 16;                 // 90112

// Int8 lattices with L % 64 == 0 that are swept by the phase kernels keep a
// copy of their state in the 2-bit class layout (N/4 bytes) after the fixed
// part of their scratch: the sweeps of a call run on that copy, which is
// packed from the int8 codes before them and unpacked into them after.
constexpr size_t kScrWork = kScrBytes;
inline bool int8_packs(int L, int enc) { return enc == 0 && L % 64 == 0; }

// Per-lattice descriptor kept in the lattice's scratch, read by the batched
// kernel.  next_sweep is advanced on the device by every path that sweeps.
struct LatDesc {
    void *state;
    int32_t L, enc;
    uint32_t key0, key1;
    uint64_t next_sweep;
};

// Lattices whose whole state fits one block's LDS run in the batched kernel:
// 8 sublattice classes of (L/2) rows x ceil(L/64) words (2 bits per site).
constexpr int kLdsMaxL = 512;
inline size_t lds_state_words(int L) { return (size_t)8 * (L / 2) * ((L / 4 + 15) / 16); }

// One launch of the batched kernel: block b advances lattice b by sweeps[b].
constexpr int kMaxBatch = 256;
struct BatchArgs {
    int count;
    uint8_t *scratch[kMaxBatch];
    uint32_t sweeps[kMaxBatch];
    // non-null: after the sweeps, lattice b's observables and tracker total
    // go to obs_out[10b ..] in k_obs_batch's layout (written by the sweep
    // kernel itself in its 512-thread word form, else by k_obs_batch)
    unsigned long long *obs_out;
};

// One phase of one sweep: phase p, displacement D = (r + 4m, 1 + 2k).
struct PhaseArgs {
    void *state;
    const uint2 *dev_tab;    // kDevTabEntries
    const uint2 *trans;      // kTransEntries
    const uint4 *trans_d;    // kTransEntries, delta form
    unsigned long long *track;  // tracker slots: block b adds its 3 sums at track[3b..3b+2]
    int L;
    int p, r, m, k;
    uint32_t key0, key1;
    uint32_t s_lo, s_hi;
    uint32_t magicW;  // ceil(2^32 / W) for W = L/64 words per class row (0 when W = 1)
};
// ceil(2^32 / W): umulhi(n, it) equals n / W (rounded down) whenever
// n (it W - 2^32) < 2^32, in particular for thread indices n < 1024 at any
// W < 2^22.
inline uint32_t magic_div(uint32_t W) { return W <= 1 ? 0u : (uint32_t)((0x100000000ull + W - 1u) / W); }

// Bound of a device-wide barrier wait in the persistent kernels: ticks of
// the device's constant-rate wall clock (100 MHz), 0.2 s.
constexpr long long kBarrierTimeoutTicks = 20000000;

// One phase of up to kWordsBatch lattices in the 2-bit class layout (int8
// ones through their packed copy), spread over many blocks per lattice:
// blocks first_block[i] .. first_block[i+1]-1 update lattice i, Q lanes per
// a-word.  Sweep iter of the series (sweep next_sweep + iter of each lattice,
// schedule computed on the device); a lattice with sweeps[i] <= iter is
// skipped.  Block b of a lattice adds its tracker sums to tracker slot b.
constexpr int kWordsBatch = 64;
constexpr int kWordsThreads = 256;
struct WordsArgs {
    int count;
    int p;
    uint32_t iter;
    uint8_t *scratch[kWordsBatch];
    uint32_t sweeps[kWordsBatch];
    uint32_t first_block[kWordsBatch + 1];
};
// Lanes per a-word for side L (fewer for larger lattices, whose words fill
// the chip anyway), and the blocks one lattice takes.
int words_lanes(int L);
inline uint32_t words_blocks(int L, int Q, int threads = kWordsThreads)
{
    const uint32_t tasks = (uint32_t)Q * (uint32_t)L * (uint32_t)L / 128u;
    return (tasks + (uint32_t)threads - 1) / (uint32_t)threads;
}
// Threads per block of the per-phase form: a multiple of 64 up to 1024
// (every block stages the tables, so larger blocks stage them fewer times).
constexpr int kWordsPhaseMaxThreads = 1024;
hipError_t launch_phase_words(const WordsArgs &a, int Q, int threads, hipStream_t s);
// desc->next_sweep += sweeps[i] for every lattice of the series.
hipError_t launch_advance_words(const WordsArgs &a, hipStream_t s);
// Persistent multi-block form: up to kWordsBatch lattices (blocks
// first_block[i] .. first_block[i+1]-1 update lattice i) for intervals x
// every sweeps in one cooperative launch, a device-wide barrier after every
// phase; lattice i runs its first sweeps[i] of them.  With records (one
// lattice, kSeriesRecord bytes each, as launch_observables writes them) the
// observables and tracker after every interval.  The barrier counter (in
// the first lattice's scratch) is cleared and the records initialised by
// kernels enqueued first.
struct WordsSeriesArgs {
    int count;
    int threads;              // block size: a multiple of 64 up to kWordsThreads
    long long barrier_ticks;  // bound of each device-wide barrier wait (device wall-clock ticks)
    uint32_t intervals, every;
    long long *records;  // null: no observables
    uint8_t *scratch[kWordsBatch];
    uint32_t sweeps[kWordsBatch];
    uint32_t first_block[kWordsBatch + 1];
};
// Blocks of the persistent launch that can be resident at once (0 when
// co-residency cannot be guaranteed: no cooperative launch); the caller then
// uses the per-phase launches.
int words_persistent_capacity(int Q, int threads);
hipError_t launch_words_series(const WordsSeriesArgs &a, int Q, hipStream_t s);
// int8 codes (row-major) <-> the 2-bit class layout, for L % 64 == 0.
hipError_t launch_pack_int8(const int8_t *src, uint32_t *dst, int L, hipStream_t s);
hipError_t launch_unpack_int8(const uint32_t *src, int8_t *dst, int L, hipStream_t s);

// Launch shape of the 2-bit phase kernel: rows of the a-class per block
// (0 = automatic) and blocks per compute unit.
struct Tuning2Bit {
    int rows_per_block;
    int blocks_per_cu;
    int waves_hint;  // >= 8: the build limited to 64 VGPRs (8 waves per SIMD)
    int persistent;  // 1: one cooperative launch per lattice_sweep call (2-bit), 0: a launch per phase
};

hipError_t launch_phase_int8(const PhaseArgs &a, hipStream_t s);
hipError_t launch_phase_2bit(const PhaseArgs &a, const Tuning2Bit &t, hipStream_t s);
// Persistent 2-bit sweeps (one cooperative launch, device-wide barrier per
// phase); hipErrorNotSupported when co-residency cannot be guaranteed.
bool persistent_2bit_supported(int L, const Tuning2Bit &t, int *grid, int *rows);
hipError_t launch_sweeps_2bit(const PhaseArgs &a, const Tuning2Bit &t, uint32_t sweeps, unsigned *counter,
                              unsigned *err, hipStream_t s);
hipError_t launch_zero_i64(unsigned long long *p, int n, hipStream_t s);
// Observable sums of the whole lattice into the observable slots (one block
// per slot, at most kMaxObsSlots blocks), then the fold of slots into the
// totals at scratch + kScrTrack (tracker) and + kScrObs (observables), or,
// with a record, into record[0..9] (tracker, 7 sums) and record[10] = the
// lattice's next sweep index (a series record, kSeriesRecord bytes).
constexpr size_t kSeriesRecord = 88;
hipError_t launch_observables(uint8_t *scratch, const void *state, int L, int encoding, hipStream_t s,
                              long long *record = nullptr);
// Batched kernel; dynamic LDS is sized for the largest L.  threads = block
// size (a multiple of 64, at most 1024; 0 = min(1024, N/16 of the largest L)).
// Map mode (section 3.2 random maps): lattices with L <= kMapMaxL, one block
// per lattice holding the codes (one byte per site), the map's mark bitmap,
// its pair list and the full threshold table in LDS.
constexpr int kMapMaxL = 256;
constexpr int kMapThreads = 512;
struct MapArgs {
    int count;
    uint8_t *scratch[kMaxBatch];
    uint32_t first_map_lo, first_map_hi, n_maps;
    int32_t nn;        // 1: nearest-neighbour partners, max(1, N/20) pairs per map
    int32_t builders;  // maps built at once (one per wave), each with its own bitmap and pair list
};
// LDS bytes one block needs for a lattice of side L with `builders` maps in flight.
inline size_t map_lds_bytes(int L, int builders)
{
    const size_t N = (size_t)L * L, pairs = N / 10 < 1 ? 1 : N / 10;
    return (size_t)kTabSize * 4 + (N + 3) / 4 * 4 + (size_t)builders * ((N + 31) / 32 * 4 + pairs * 4);
}
// Dynamic LDS a map block may use (160 KiB per workgroup, less the static reduction buffer).
constexpr size_t kMapLdsMax = 160 * 1024 - 1024;
hipError_t launch_map_steps(const MapArgs &a, int max_L, hipStream_t s);
hipError_t init_map_kernel_attributes();

// Penalty mode: one half-sweep (checkerboard colour c) of an int8 lattice.
struct MuArgs {
    int8_t *state;
    const uint32_t *tab;   // kMuTabSize thresholds (scratch + kScrMuTab)
    unsigned long long *track;  // per-block tracker slots
    int L, colour;
    uint32_t key0, key1, s_lo, s_hi;
};
hipError_t launch_mu_half(const MuArgs &a, hipStream_t s);

// One-time kernel set-up (dynamic LDS limits); called before the first launch.
hipError_t init_kernel_attributes();
// Batched sweeps with each lattice resident in LDS.  word = every lattice of
// the batch has L % 64 == 0 (word-parallel form); otherwise the per-site form.
hipError_t launch_sweep_lds(const BatchArgs &a, int max_L, int threads, bool word, hipStream_t s);
// desc->next_sweep += sweeps (after host-scheduled phase launches).
hipError_t launch_advance(LatDesc *desc, uint32_t sweeps, hipStream_t s);
// Observables of `count` lattices in one launch: out[10*b .. 10*b+9] =
// (tracker nD, nV, nJ, then the 7 sums) of lattice b.
hipError_t launch_observables_batch(const BatchArgs &a, unsigned long long *out, hipStream_t s);

}  // namespace lat
