// Library-internal declarations shared by the host sources (lattice_api.cpp,
// server.cpp).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <string>

#include "../../include/lattice.h"
#include "kernels.h"

// How a lattice is swept (chosen at create from L and the encoding):
//   kPathLds    one block holds the whole lattice in LDS for all the sweeps of
//               a launch (batch.hip); by default L <= 256 when L % 64 == 0,
//               else L <= 512;
//   kPathWords  many blocks per lattice, Q lanes per a-word, schedule
//               computed on the device (words.hip): one persistent launch
//               per call up to L = 1024, else one launch per phase;
//               L % 64 == 0, L <= 2048;
//   kPathPhase  one launch per phase, one thread per a-word (phase.hip).
// Int8 lattices with L % 64 == 0 on the last two paths are swept on a 2-bit
// copy in their scratch (packed before the sweeps of a call, unpacked after).
enum : int { kPathLds = 0, kPathWords = 1, kPathPhase = 2 };

struct lattice {
    int L = 0, enc = 0;
    int64_t N = 0, Q = 0, Nc = 0;
    double n = 0, Delta = 0, V = 0, J = 0, T = 1;
    uint64_t seed = 0, start_sweep = 0, done = 0;
    void *d_state = nullptr;
    uint8_t *d_scratch = nullptr;
    hipStream_t stream = nullptr;
    lat::Tuning2Bit tuning{0, 0, 0, 0};
    int path = kPathLds;
    bool packed = false;  // int8 swept on the 2-bit copy at scratch + kScrWork
    // set once a persistent launch has swept it, so that reads check the
    // device-wide barrier's time-out flag
    bool ran_persistent = false;
    uint32_t magic = 0;
};

namespace lat {
namespace detail {

int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
// fail() for exception handlers: records "what: msg" without throwing (if
// even that string cannot be allocated, a fixed message is kept instead).
int fail_nothrow(int code, const char *what, const char *msg) noexcept;
bool live(const lattice *h);

// Runs the body of a C-ABI entry point so that no C++ exception crosses the
// ABI: host memory exhaustion (std::bad_alloc) becomes LAT_ENOMEM, anything
// else (a thread that cannot start, a container error) LAT_EHIP, each with a
// message for lattice_last_error().
template <class F>
int guarded(const char *what, F &&body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail_nothrow(LAT_ENOMEM, what, "out of host memory");
    } catch (const std::exception &e) {
        return fail_nothrow(LAT_EHIP, what, e.what());
    } catch (...) {
        return fail_nothrow(LAT_EHIP, what, "unknown exception");
    }
}
// Advance lattices resident in LDS; lattice i by sweeps[i] (null: `uniform`).
// tune = false: no autotuning launches (the tuned or default block size),
// as needed under stream capture.  obs_dev non-null: then also write the
// lattices' observables into obs_dev (10 int64 each, as
// enqueue_observables_batch), from LDS at the end of the 512-thread
// word-form launch or by a separate launch after the other forms.
int enqueue_lds_sweeps(lattice *const *hs, int32_t count, const uint32_t *sweeps, uint32_t uniform,
                       hipStream_t stream, bool tune = true, unsigned long long *obs_dev = nullptr);
// One batched observables launch per 256 lattices into dev (10 int64 each).
int enqueue_observables_batch(lattice *const *hs, int32_t count, unsigned long long *dev, hipStream_t stream);
// Lattices on the off-chip paths (words, phase): lattice i by sweeps[i]
// (null: `uniform`); int8 ones are packed before and unpacked after.
// convert = false: packed lattices are already on (and stay on) their copy.
// persistent = false: the multi-block lattices take one launch per phase,
// never the cooperative persistent launch, whose blocks must all be resident
// at once (callers whose other streams run kernels at the same time, like
// the server, would otherwise leave it waiting for compute units).
int enqueue_offchip_sweeps(lattice *const *hs, int32_t count, const uint32_t *sweeps, uint32_t uniform,
                           hipStream_t stream, bool convert = true, bool persistent = true);
// Lattices of the multi-block path as persistent launches: lattice i by
// sweeps[i] (null: `every`) with intervals = 1 and no records, or, with
// records, an observation series of one lattice: intervals x every sweeps, a
// kSeriesRecord record after each interval.  *ran = false (nothing
// enqueued) when the persistent form is off (by default above L = 1024;
// LATTICE_WORDS_PERSISTENT=0|1 overrides) or cannot be launched here; the
// caller then uses the per-phase launches.  Packed int8 lattices must
// already be on their 2-bit copy.
int enqueue_words_persistent(lattice *const *hs, int32_t count, const uint32_t *sweeps, uint32_t intervals,
                             uint32_t every, long long *records, hipStream_t stream, bool *ran);
// Checks of lat_params (geometry, finite couplings, T > 0, the charge target
// of eq. 2); writes the target charge and the charged count.
int validate_params(const lat_params *p, int64_t *Q, int64_t *Nc);
// The lattice has run a persistent kernel, whose bounded device-wide barrier
// flags a time-out in its error word.
bool barrier_may_time_out(const lattice *h);
// v = (tracker nD, nV, nJ, sum S, sum S^2, bonds SS, bonds ss, M, M_st, C_st).
void fill_obs(const lattice *h, const int64_t *v, lat_obs *out);

// Launch-shape autotuner for the batched kernel.  For every (largest L,
// batch size) it tries each candidate block size on one real call, timed with
// HIP events on the call's stream, then keeps the fastest per site update.
// The chain does not depend on the launch shape, so tuning runs real work.
// LATTICE_BATCH_THREADS=<n> pins the block size instead.
int batch_threads_for(int max_L, int count, bool word, hipStream_t stream, hipEvent_t *start, hipEvent_t *stop,
                      int *slot);
void batch_threads_done(int slot, double site_updates);

}  // namespace detail
}  // namespace lat
