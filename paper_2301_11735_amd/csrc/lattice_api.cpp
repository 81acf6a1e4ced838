// Host side of liblattice.so: the C-ABI of include/lattice.h.
//
// Parameter checks and the charge target (eq. 2), the stage-1 initial
// configuration (section 3.1), the FP64 Metropolis threshold table (section
// 3.1, eq. 3), the per-sweep schedule of non-interacting pairs (section 3.2)
// and the layout conversion between canonical codes and the device encodings.
// All sweep and reduction work runs in the kernels of phase.hip, obs.hip and
// batch.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <mutex>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lattice.h"
#include "internal.h"
#include "kernels.h"
#include "philox.h"

using namespace lat;
using namespace lat::detail;

namespace {

constexpr uint32_t kMagic = 0x1A771CEu;
constexpr int kMaxL = 32768;

thread_local std::string g_err;
thread_local const char *g_err_fixed = nullptr;  // set when g_err could not be formatted

}  // namespace

namespace lat {
namespace detail {

int fail(int code, const std::string &msg)
{
    g_err_fixed = nullptr;
    g_err = msg;
    return code;
}

int fail_nothrow(int code, const char *what, const char *msg) noexcept
{
    try {
        g_err_fixed = nullptr;
        g_err = std::string(what) + ": " + msg;
    } catch (...) {
        g_err_fixed = code == LAT_ENOMEM ? "out of host memory" : "error (its message could not be stored)";
    }
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(LAT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool live(const lattice *h) { return h != nullptr && h->magic == kMagic; }

}  // namespace detail
}  // namespace lat

namespace {

bool valid_geometry(int32_t L, int32_t enc)
{
    if (L < 4 || L > kMaxL) return false;
    if (enc == LAT_ENC_INT8) return L % 4 == 0;
    if (enc == LAT_ENC_2BIT) return L % 64 == 0;
    return false;
}

// Eq. (2) made an integer: Q nearest nN with the parity of the charged count
// (ties to the smaller); without a requested count, Nc = max(N/4, |Q|).
int charge_target(int32_t L, double n, int64_t n_req, int64_t *Q_out, int64_t *Nc_out)
{
    const int64_t N = (int64_t)L * L;
    const double target = n * (double)N;
    if (!std::isfinite(target) || std::fabs(target) > (double)N) return fail(LAT_EINVAL, "n must satisfy |n| <= 1");
    const int64_t nc0 = n_req >= 0 ? n_req : N / 4;
    if (nc0 > N) return fail(LAT_EINVAL, "n_charged exceeds N");
    const int64_t parity = nc0 & 1;
    int64_t lo = (int64_t)std::floor(target);
    if ((lo & 1) != parity) lo -= 1;  // two's complement: & 1 is the parity for negatives too
    const int64_t hi = lo + 2;
    const int64_t Q = ((double)hi - target < target - (double)lo) ? hi : lo;
    int64_t Nc = nc0;
    if (std::llabs(Q) > nc0) {
        if (n_req >= 0) return fail(LAT_EINVAL, "|Q| exceeds the requested number of charged sites");
        Nc = std::llabs(Q);
    }
    if (Nc > N) return fail(LAT_EINVAL, "no charge target fits the lattice");
    *Q_out = Q;
    *Nc_out = Nc;
    return LAT_OK;
}

// Stage 1 of section 3.1: site i gets key (w0 << 32 | w1) of Philox counter
// (0, 0x200, i, 0); the N+ smallest (key, i) become +1, the next N- become -1,
// the others are spins with sigma from bit 0 of w2.  Selection (two
// nth_element passes) gives the same sets as a full sort.
void seeded_init(int32_t L, uint64_t seed, int64_t n_plus, int64_t n_minus, std::vector<int8_t> &codes)
{
    const int64_t N = (int64_t)L * L;
    struct Key {
        uint64_t k;
        uint32_t i;
        bool operator<(const Key &o) const { return k != o.k ? k < o.k : i < o.i; }
    };
    std::vector<Key> keys((size_t)N);
    codes.assign((size_t)N, 0);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (N < (1 << 16)) nt = 1;
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nt; ++t) {
        pool.emplace_back([&, t] {
            const int64_t b = N * t / nt, e = N * (t + 1) / nt;
            for (int64_t i = b; i < e; ++i) {
                const u32x4 w = philox4x32_10(0u, kDomInit, (uint32_t)i, 0u, k0, k1);
                keys[(size_t)i] = Key{((uint64_t)w.x << 32) | w.y, (uint32_t)i};
                codes[(size_t)i] = (int8_t)(w.z & 1u);
            }
        });
    }
    for (auto &th : pool) th.join();
    const int64_t nc = n_plus + n_minus;
    if (nc > 0) {
        if (nc < N) std::nth_element(keys.begin(), keys.begin() + nc, keys.end());
        if (n_plus > 0 && n_plus < nc) std::nth_element(keys.begin(), keys.begin() + n_plus, keys.begin() + nc);
        for (int64_t r = 0; r < nc; ++r) codes[keys[(size_t)r].i] = (int8_t)(r < n_plus ? 2 : 3);
    }
}

// Section 3.1: classical Metropolis acceptance for every energy-change triple,
// dE = Delta*nD + V*nV + 0.25*J*nJ (eq. 3) in FP64; "always" for dE <= 0.
void build_threshold_table(double Delta, double V, double J, double T, std::vector<uint32_t> &tab)
{
    tab.assign(kTabSize, 0u);
    for (int nD = -2; nD <= 2; ++nD)
        for (int nV = -16; nV <= 16; ++nV)
            for (int nJ = -16; nJ <= 16; ++nJ) {
                const double dE = Delta * nD + V * nV + 0.25 * J * nJ;
                uint32_t t;
                if (dE <= 0.0) {
                    t = 0xFFFFFFFFu;
                } else {
                    const double f = std::floor(std::exp(-dE / T) * 4294967296.0);
                    t = f >= 4294967294.0 ? 0xFFFFFFFEu : (uint32_t)f;
                }
                tab[(size_t)(nD + 2) * (kTabV * kTabJ) + (size_t)(nV + 16) * kTabJ + (size_t)(nJ + 16)] = t;
            }
}

// Packed triple an accepted move adds to the per-thread tracker.
uint32_t packed_triple(int nD, int nV, int nJ)
{
    return (1u << 27) | ((uint32_t)(nD + 2) << 20) | ((uint32_t)(nV + 16) << 10) | (uint32_t)(nJ + 16);
}

uint32_t threshold_of(const std::vector<uint32_t> &tab, int nD, int nV, int nJ)
{
    return tab[(size_t)(nD + 2) * (kTabV * kTabJ) + (size_t)(nV + 16) * kTabJ + (size_t)(nJ + 16)];
}

// Device threshold table: the reachable triples only (regions in kernels.h),
// each entry paired with its packed tracker triple.
void build_device_table(const std::vector<uint32_t> &tab, std::vector<uint32_t> &dev)
{
    dev.assign(2 * (size_t)kDevTabEntries, 0u);
    auto put = [&](size_t i, int nD, int nV, int nJ) {
        dev[2 * i] = threshold_of(tab, nD, nV, nJ);
        dev[2 * i + 1] = packed_triple(nD, nV, nJ);
    };
    for (int s = 0; s < 3; ++s)
        for (int nV = -8; nV <= 8; ++nV)
            for (int nJ = -8; nJ <= 8; ++nJ)
                put((size_t)s * kDevSlice + (size_t)(nV + 8) * 17 + (size_t)(nJ + 8), 2 * s - 2, nV, nJ);
    for (int v = -16; v <= 16; ++v) {
        put((size_t)kDevVLine + (size_t)(v + 16), 0, v, 0);
        put((size_t)kDevJLine + (size_t)(v + 16), 0, 0, v);
    }
}

// Transition table of section 3.1's coupled-pair move.  For pair state
// st = code_a | code_b << 2 and choice j < k_q: the j-th configuration of the
// same-charge set in the paper's listing order,
//   q=+1: (2,0) (2,1) (0,2) (1,2)
//   q= 0: (2,3) (3,2) (0,0) (1,1) (0,1) (1,0)
//   q=-1: (3,0) (3,1) (0,3) (1,3),
// and the coefficients that turn the neighbour sums (each offset by +4) into
// the device-table index of the move's (nD, nV, nJ).  Since the pair keeps its
// charge, dS_a + dS_b = 0 and the +4 offsets of the charge sums cancel; the
// spin offsets 4*(dsig_a + dsig_b) are folded into C.  The frozen states
// (|q| = 2) get one null move.  trans_d is the delta form (4 words an entry).
void build_transition_table(std::vector<uint32_t> &trans, std::vector<uint32_t> &trans_d)
{
    static const int kS[4] = {0, 0, 1, -1}, kG[4] = {1, -1, 0, 0};
    static const int kPlus1[4][2] = {{2, 0}, {2, 1}, {0, 2}, {1, 2}};
    static const int kZero[6][2] = {{2, 3}, {3, 2}, {0, 0}, {1, 1}, {0, 1}, {1, 0}};
    static const int kMinus1[4][2] = {{3, 0}, {3, 1}, {0, 3}, {1, 3}};
    trans.assign(2 * (size_t)kTransEntries, 0u);
    trans_d.assign(4 * (size_t)kTransEntries, 0u);
    auto i8 = [](int v) { return (uint32_t)(uint8_t)(int8_t)v; };
    for (int st = 0; st < 16; ++st) {
        const int ca = st & 3, cb = st >> 2, q = kS[ca] + kS[cb];
        const int (*set)[2] = q == 1 ? kPlus1 : (q == 0 ? kZero : (q == -1 ? kMinus1 : nullptr));
        const int kq = set ? (q == 0 ? 6 : 4) : 1;
        for (int j = 0; j < kq; ++j) {
            const int a1 = set ? set[j][0] : ca, b1 = set ? set[j][1] : cb;
            const int dSa = kS[a1] - kS[ca], dSb = kS[b1] - kS[cb];
            const int dGa = kG[a1] - kG[ca], dGb = kG[b1] - kG[cb];
            const int nD = kS[a1] * kS[a1] + kS[b1] * kS[b1] - kS[ca] * kS[ca] - kS[cb] * kS[cb];
            uint32_t coef;
            int C;
            if (dSa == 2 || dSa == -2) {  // charge swap: V line, nJ = 0
                coef = i8(dSa) | (i8(dSb) << 8);
                C = kDevVLine + 16;
            } else if (dGa == 2 || dGa == -2 || dGb == 2 || dGb == -2) {  // spin change: J line, nV = 0
                coef = (i8(dGa) << 16) | (i8(dGb) << 24);
                C = kDevJLine + 16 - 4 * (dGa + dGb);
            } else {  // |dS|, |dsig| <= 1: slice nD/2 + 1
                coef = i8(17 * dSa) | (i8(17 * dSb) << 8) | (i8(dGa) << 16) | (i8(dGb) << 24);
                C = (nD / 2 + 1) * kDevSlice + 8 * 17 + 8 - 4 * (dGa + dGb);
            }
            trans[2 * (size_t)(st * 6 + j)] = coef;
            trans[2 * (size_t)(st * 6 + j) + 1] = (uint32_t)C | ((uint32_t)(a1 | (b1 << 2)) << 16);
            uint32_t *d = &trans_d[4 * (size_t)(st * 6 + j)];
            d[0] = coef;
            d[1] = (uint32_t)C;
            d[2] = (uint32_t)(a1 ^ ca) * 0x5555u | ((uint32_t)(b1 ^ cb) * 0x5555u) << 16;
            d[3] = 0u;
        }
    }
}

Tuning2Bit tuning_from_env()
{
    Tuning2Bit t{0, 0, 0, 0};
    if (const char *v = std::getenv("LATTICE_2BIT_ROWS")) t.rows_per_block = std::atoi(v);
    if (const char *v = std::getenv("LATTICE_2BIT_BLOCKS_PER_CU")) t.blocks_per_cu = std::atoi(v);
    if (const char *v = std::getenv("LATTICE_2BIT_WAVES")) t.waves_hint = std::atoi(v);
    if (const char *v = std::getenv("LATTICE_PERSISTENT")) t.persistent = std::atoi(v);
    return t;
}

// Canonical row-major codes <-> device encoding.
void to_device_layout(int32_t L, int32_t enc, const std::vector<int8_t> &codes, std::vector<uint8_t> &out)
{
    const size_t N = (size_t)L * L;
    if (enc == LAT_ENC_INT8) {
        out.assign((const uint8_t *)codes.data(), (const uint8_t *)codes.data() + N);
        return;
    }
    const size_t W = (size_t)L / 64, H = (size_t)L / 2, csz = H * W;
    std::vector<uint32_t> words(N / 16, 0u);
    for (size_t y = 0; y < (size_t)L; ++y)
        for (size_t x = 0; x < (size_t)L; ++x) {
            const size_t c = 4 * (y & 1) + (x & 3), X = x >> 2, Y = y >> 1;
            words[c * csz + Y * W + (X >> 4)] |= (uint32_t)(codes[y * L + x] & 3) << (2 * (X & 15));
        }
    out.resize(N / 4);
    std::memcpy(out.data(), words.data(), N / 4);
}

void from_device_layout(int32_t L, int32_t enc, const std::vector<uint8_t> &dev, int8_t *codes)
{
    const size_t N = (size_t)L * L;
    if (enc == LAT_ENC_INT8) {
        std::memcpy(codes, dev.data(), N);
        return;
    }
    const size_t W = (size_t)L / 64, H = (size_t)L / 2, csz = H * W;
    const uint32_t *words = (const uint32_t *)dev.data();
    for (size_t y = 0; y < (size_t)L; ++y)
        for (size_t x = 0; x < (size_t)L; ++x) {
            const size_t c = 4 * (y & 1) + (x & 3), X = x >> 2, Y = y >> 1;
            codes[y * L + x] = (int8_t)((words[c * csz + Y * W + (X >> 4)] >> (2 * (X & 15))) & 3u);
        }
}

// Schedule of sweep s (section 3.2: non-interacting pairs, long-range
// partners): r in {1,2,3}; phase p has D_p = (r + 4 m_p, 1 + 2 k_p).
struct Schedule {
    int r, m[4], k[4];
};

Schedule sweep_schedule(int32_t L, uint64_t seed, uint64_t s)
{
    uint32_t Wd[12];
    for (uint32_t t = 0; t < 3; ++t) {
        const u32x4 w = philox4x32_10((uint32_t)s, kDomSchedule, t, (uint32_t)(s >> 32), (uint32_t)seed,
                                      (uint32_t)(seed >> 32));
        Wd[4 * t] = w.x;
        Wd[4 * t + 1] = w.y;
        Wd[4 * t + 2] = w.z;
        Wd[4 * t + 3] = w.w;
    }
    Schedule sc;
    sc.r = 1 + (int)(((uint64_t)(Wd[0] >> 8) * 3u) >> 24);
    for (int p = 0; p < 4; ++p) {
        sc.m[p] = (int)mulhi_u32(Wd[1 + 2 * p], (uint32_t)(L / 4));
        sc.k[p] = (int)mulhi_u32(Wd[2 + 2 * p], (uint32_t)(L / 2));
    }
    return sc;
}

}  // namespace

namespace lat {
namespace detail {

namespace {

// The buffer and encoding the off-chip kernels sweep: the lattice's own
// state, or the 2-bit copy of a packed int8 lattice.
void *swept_state(const lattice *h) { return h->packed ? (void *)(h->d_scratch + kScrWork) : h->d_state; }
int swept_enc(const lattice *h) { return h->packed ? LAT_ENC_2BIT : h->enc; }

// Host-scheduled path: four phase launches per sweep, then the device-side
// sweep counter is advanced to match.
int enqueue_phase_sweeps(lattice *h, uint32_t sweeps, hipStream_t stream)
{
    PhaseArgs a{};
    a.state = swept_state(h);
    a.dev_tab = (const uint2 *)(h->d_scratch + kScrDevTab);
    a.trans = (const uint2 *)(h->d_scratch + kScrTrans);
    a.trans_d = (const uint4 *)(h->d_scratch + kScrTransD);
    a.track = (unsigned long long *)(h->d_scratch + kScrSlots);
    a.L = h->L;
    a.magicW = magic_div((uint32_t)h->L >> 6);
    a.key0 = (uint32_t)h->seed;
    a.key1 = (uint32_t)(h->seed >> 32);
    const int enc = swept_enc(h);
    uint32_t left = sweeps;
    if (enc == LAT_ENC_2BIT && h->tuning.persistent) {
        // one cooperative launch per chunk; the barrier counter stays far below 2^32
        constexpr uint32_t kChunk = 65536;
        while (left > 0) {
            const uint32_t n = std::min(left, kChunk);
            const uint64_t s = h->start_sweep + h->done + (sweeps - left);
            a.s_lo = (uint32_t)s;
            a.s_hi = (uint32_t)(s >> 32);
            const hipError_t e = launch_sweeps_2bit(a, h->tuning, n, (unsigned *)(h->d_scratch + kScrBarrier),
                                                    (unsigned *)(h->d_scratch + kScrErr), stream);
            if (e == hipErrorNotSupported) break;  // no co-residency guarantee: per-phase launches below
            if (e != hipSuccess) return hip_fail(e, "persistent sweep launch");
            left -= n;
        }
    }
    for (uint32_t i = sweeps - left; i < sweeps; ++i) {
        const uint64_t s = h->start_sweep + h->done + i;
        const Schedule sc = sweep_schedule(h->L, h->seed, s);
        a.s_lo = (uint32_t)s;
        a.s_hi = (uint32_t)(s >> 32);
        a.r = sc.r;
        for (int p = 0; p < 4; ++p) {
            a.p = p;
            a.m = sc.m[p];
            a.k = sc.k[p];
            const hipError_t e =
                enc == LAT_ENC_INT8 ? launch_phase_int8(a, stream) : launch_phase_2bit(a, h->tuning, stream);
            if (e != hipSuccess) return hip_fail(e, "phase kernel launch");
        }
    }
    if (sweeps > 0) {
        const hipError_t e = launch_advance((LatDesc *)(h->d_scratch + kScrDesc), sweeps, stream);
        if (e != hipSuccess) return hip_fail(e, "advance kernel launch");
    }
    h->done += sweeps;
    return LAT_OK;
}

// Threads per block of the per-phase word kernel (LATTICE_WORDS_BLOCK: a
// multiple of 64 up to 1024).
int words_phase_threads()
{
    const char *v = std::getenv("LATTICE_WORDS_BLOCK");
    const int want = v ? std::atoi(v) : 0;
    return want >= 64 && want <= kWordsPhaseMaxThreads && want % 64 == 0 ? want : kWordsThreads;
}

// Multi-block word path: lattices in groups of up to kWordsBatch per launch,
// one launch per phase of every sweep of the series (the lattice i of a
// group skips the sweeps past sweeps[i]), then the device sweep counters
// are advanced.  Q (lanes per a-word) is chosen by the largest L of the
// group; every lattice's blocks must fit its kMaxSlots tracker slots.
int enqueue_words_sweeps(lattice *const *hs, int32_t count, const uint32_t *sweeps, uint32_t uniform,
                         hipStream_t stream)
{
    for (int32_t b = 0; b < count; b += kWordsBatch) {
        WordsArgs a{};
        a.count = std::min<int32_t>(kWordsBatch, count - b);
        int max_L = 0;
        for (int i = 0; i < a.count; ++i) max_L = std::max(max_L, hs[b + i]->L);
        int Q = words_lanes(max_L);
        // LATTICE_WORDS_PHASE_LANES (1, 2, 4 or 8) overrides the lanes per a-word
        if (const char *v = std::getenv("LATTICE_WORDS_PHASE_LANES")) {
            const int want = std::atoi(v);
            if (want == 1 || want == 2 || want == 4 || want == 8) Q = want;
        }
        const int threads = words_phase_threads();
        uint32_t blocks = 0, most = 0;
        for (int i = 0; i < a.count; ++i) {
            const lattice *h = hs[b + i];
            const uint32_t nb = words_blocks(h->L, Q, threads);
            if (nb > (uint32_t)kMaxSlots) return fail(LAT_EINVAL, "lattice too large for the multi-block word kernel");
            a.scratch[i] = h->d_scratch;
            a.sweeps[i] = sweeps ? sweeps[b + i] : uniform;
            a.first_block[i] = blocks;
            blocks += nb;
            most = std::max(most, a.sweeps[i]);
        }
        a.first_block[a.count] = blocks;
        if (most == 0) continue;
        for (uint32_t it = 0; it < most; ++it) {
            a.iter = it;
            for (int p = 0; p < 4; ++p) {
                a.p = p;
                const hipError_t e = launch_phase_words(a, Q, threads, stream);
                if (e != hipSuccess) return hip_fail(e, "word phase kernel launch");
            }
        }
        const hipError_t e = launch_advance_words(a, stream);
        if (e != hipSuccess) return hip_fail(e, "advance kernel launch");
        for (int i = 0; i < a.count; ++i) hs[b + i]->done += a.sweeps[i];
    }
    return LAT_OK;
}

}  // namespace

constexpr int kWordsPersistentMaxL = 1024;

namespace {

// Resident-block capacity of the persistent word kernel per (device, Q),
// looked up once.
int words_capacity(int Q, int threads)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(dev, Q, threads);
    auto it = cache.find(key);
    if (it == cache.end()) it = cache.emplace(key, words_persistent_capacity(Q, threads)).first;
    return it->second;
}

// Bound of each device-wide barrier wait of the persistent word kernel:
// kBarrierTimeoutTicks unless LATTICE_BARRIER_TICKS asks for another
// (non-negative) count; tests use a tiny one to force the time-out path,
// whose kernels still end normally (a wait that times out flags the state
// invalid and goes on).
long long words_barrier_ticks()
{
    if (const char *v = std::getenv("LATTICE_BARRIER_TICKS")) {
        const long long want = std::atoll(v);
        if (want >= 0) return want;
    }
    return kBarrierTimeoutTicks;
}

// Block size of the persistent word kernel: 256 threads unless
// LATTICE_WORDS_SERIES_BLOCK asks for another multiple of 64 up to 256
// (smaller blocks spread a lattice over more compute units).
int words_series_threads()
{
    if (const char *v = std::getenv("LATTICE_WORDS_SERIES_BLOCK")) {
        const int want = std::atoi(v);
        if (want >= 64 && want <= kWordsThreads && want % 64 == 0) return want;
    }
    return kWordsThreads;
}

}  // namespace

int enqueue_words_persistent(lattice *const *hs, int32_t count, const uint32_t *sweeps, uint32_t intervals,
                             uint32_t every, long long *records, hipStream_t stream, bool *ran)
{
    *ran = false;
    if (count <= 0 || intervals == 0 || every == 0) return LAT_OK;
    int max_L = 0;
    for (int32_t i = 0; i < count; ++i) {
        if (hs[i]->path != kPathWords) return LAT_OK;
        max_L = std::max(max_L, hs[i]->L);
    }
    // default: on up to L = 1024, where it measured faster than one launch
    // per phase (13.2 against 21.9 us a sweep at L = 512, 23.0 against
    // 24.7 us at L = 1024); above, its device-coherent loads, which no
    // compute unit's cache serves, cost more than the launches they save
    // (43 against 28 us at L = 2048).  A series with observables every sweep
    // takes its records from the tracked moves in this form (no pass over
    // the lattice, no extra barrier): 25.6 us a sweep at L = 1024, against
    // 34.6 us with launches per phase and a reduction launch per interval.
    // LATTICE_WORDS_PERSISTENT=0|1 overrides.
    const char *v = std::getenv("LATTICE_WORDS_PERSISTENT");
    if (v ? std::atoi(v) == 0 : max_L > kWordsPersistentMaxL) return LAT_OK;
    if (records && count != 1) return fail(LAT_EINVAL, "an observation series holds one lattice");
    // lanes per a-word: 8 up to L = 512 and 2 above.  This form's
    // device-coherent loads set its pace, and fewer lanes per word load fewer
    // words in all: at L = 1024 a sweep with its observables took 26.9, 29.6
    // and 35.5 us with 2, 4 and 8 lanes (at L = 512, 17-19 us with any of
    // them); at L = 2048, 43 and 78 us with 2 and 4.  LATTICE_WORDS_LANES
    // (1, 2, 4 or 8) overrides.  Blocks of 256 threads: 128 and 64 measured
    // slower at L = 512 and 1024 (more blocks meet at every barrier).
    int Q = max_L <= 512 ? 8 : 2;
    if (const char *q = std::getenv("LATTICE_WORDS_LANES")) {
        const int want = std::atoi(q);
        if (want == 1 || want == 2 || want == 4 || want == 8) Q = want;
    }
    const int threads = words_series_threads();
    const int capacity = words_capacity(Q, threads);
    if (capacity <= 0) return LAT_OK;
    // the barrier counter counts blocks x barriers: at most 2^20 barriers per
    // launch keeps it below 2^32 for any resident grid
    constexpr uint64_t kMaxBarriers = 1u << 20;
    const uint64_t per_interval = 4ull * every;
    if (per_interval > kMaxBarriers && records) return LAT_OK;  // such intervals take the per-phase launches
    const uint32_t sweeps_cap = (uint32_t)(kMaxBarriers / 4);
    const uint32_t intervals_cap = records ? (uint32_t)std::max<uint64_t>(1, kMaxBarriers / per_interval) : 1u;

    // lattices in launches of at most kWordsBatch, each with its share of the
    // resident blocks
    for (int32_t g0 = 0; g0 < count; g0 += kWordsBatch) {
        const int32_t n = std::min<int32_t>(kWordsBatch, count - g0);
        const uint32_t share = std::max<uint32_t>(1, (uint32_t)capacity / (uint32_t)n);
        uint32_t nb[kWordsBatch];
        uint32_t total = 0;
        for (int32_t i = 0; i < n; ++i) {
            nb[i] = std::min<uint32_t>({words_blocks(hs[g0 + i]->L, Q, threads), share, (uint32_t)kMaxSlots});
            total += nb[i];
        }
        if (total > (uint32_t)capacity) return *ran ? fail(LAT_EHIP, "persistent word launch does not fit") : LAT_OK;
        if (records) {
            lattice *h = hs[g0];
            for (uint32_t k = 0; k < intervals; k += intervals_cap) {
                WordsSeriesArgs a{};
                a.count = 1;
                a.threads = threads;
                a.barrier_ticks = words_barrier_ticks();
                a.intervals = std::min(intervals_cap, intervals - k);
                a.every = every;
                a.records = records + (kSeriesRecord / 8) * (size_t)k;
                a.scratch[0] = h->d_scratch;
                a.sweeps[0] = a.intervals * every;
                a.first_block[0] = 0;
                a.first_block[1] = nb[0];
                const hipError_t e = launch_words_series(a, Q, stream);
                if (e != hipSuccess) return hip_fail(e, "persistent word kernel launch");
                h->done += (uint64_t)a.sweeps[0];
            }
            h->ran_persistent = true;
            *ran = true;
            continue;
        }
        uint32_t most = 0;
        for (int32_t i = 0; i < n; ++i) most = std::max(most, sweeps ? sweeps[g0 + i] : every);
        for (uint32_t c = 0; c < most; c += sweeps_cap) {
            WordsSeriesArgs a{};
            a.threads = threads;
            a.barrier_ticks = words_barrier_ticks();
            a.intervals = 1;
            a.every = 0;
            uint32_t blocks = 0;
            for (int32_t i = 0; i < n; ++i) {
                const uint32_t want = sweeps ? sweeps[g0 + i] : every;
                const uint32_t k = want > c ? std::min(sweeps_cap, want - c) : 0u;
                if (k == 0) continue;
                a.scratch[a.count] = hs[g0 + i]->d_scratch;
                a.sweeps[a.count] = k;
                a.first_block[a.count] = blocks;
                blocks += nb[i];
                a.every = std::max(a.every, k);
                ++a.count;
                hs[g0 + i]->done += k;
                hs[g0 + i]->ran_persistent = true;
            }
            a.first_block[a.count] = blocks;
            if (a.count == 0) continue;
            const hipError_t e = launch_words_series(a, Q, stream);
            if (e != hipSuccess) return hip_fail(e, "persistent word kernel launch");
        }
        *ran = true;
    }
    return LAT_OK;
}

int enqueue_offchip_sweeps(lattice *const *hs, int32_t count, const uint32_t *sweeps, uint32_t uniform,
                           hipStream_t stream, bool convert, bool persistent)
{
    auto n_of = [&](int32_t i) { return sweeps ? sweeps[i] : uniform; };
    for (int32_t i = 0; i < count && convert; ++i) {
        if (!hs[i]->packed || n_of(i) == 0) continue;
        const hipError_t e = launch_pack_int8((const int8_t *)hs[i]->d_state,
                                              (uint32_t *)(hs[i]->d_scratch + kScrWork), hs[i]->L, stream);
        if (e != hipSuccess) return hip_fail(e, "int8 pack launch");
    }
    std::vector<lattice *> words;
    std::vector<uint32_t> words_n;
    for (int32_t i = 0; i < count; ++i) {
        if (hs[i]->path == kPathWords) {
            words.push_back(hs[i]);
            words_n.push_back(n_of(i));
        } else {
            const int rc = enqueue_phase_sweeps(hs[i], n_of(i), stream);
            if (rc) return rc;
        }
    }
    if (!words.empty()) {
        bool ran = false;
        int rc = persistent ? enqueue_words_persistent(words.data(), (int32_t)words.size(), words_n.data(), 1, 1,
                                                       nullptr, stream, &ran)
                            : LAT_OK;
        if (rc == LAT_OK && !ran)
            rc = enqueue_words_sweeps(words.data(), (int32_t)words.size(), words_n.data(), 0, stream);
        if (rc) return rc;
    }
    for (int32_t i = 0; i < count && convert; ++i) {
        if (!hs[i]->packed || n_of(i) == 0) continue;
        const hipError_t e = launch_unpack_int8((const uint32_t *)(hs[i]->d_scratch + kScrWork),
                                                (int8_t *)hs[i]->d_state, hs[i]->L, stream);
        if (e != hipSuccess) return hip_fail(e, "int8 unpack launch");
    }
    return LAT_OK;
}

// ---- autotuner for the batched kernel's block size ----
namespace {

struct TuneEntry {
    std::vector<int> candidates;
    std::vector<double> ns_per_update;  // < 0: not measured yet
    std::vector<double> in_flight;      // > 0: site updates of a timed launch not yet read;
                                        // < 0: handed out, not yet enqueued
    std::vector<hipEvent_t> start, stop;
    int best = -1;
};

using TuneKey = std::pair<int, int>;  // (max L | word form << 20, batch size rounded up to a power of 2)
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;
std::vector<std::pair<TuneKey, int>> g_tune_slots;  // (shape, candidate) of each timed launch handed out

int pinned_batch_threads()
{
    const char *v = std::getenv("LATTICE_BATCH_THREADS");
    return v ? std::atoi(v) : 0;
}

TuneKey tune_key(int max_L, int count, bool word)
{
    int bucket = 1;
    while (bucket < count) bucket *= 2;
    return std::make_pair(max_L | (word ? 1 << 20 : 0), bucket);
}

// Reads the timed launches of a shape that have completed (never waits), and
// picks the fastest candidate once all are measured.  Caller holds g_tune_mu.
void harvest(TuneEntry &t)
{
    bool all = true;
    for (size_t i = 0; i < t.candidates.size(); ++i) {
        if (t.in_flight[i] > 0) {
            const hipError_t q = hipEventQuery(t.stop[i]);
            if (q == hipErrorNotReady) {
                all = false;
                continue;
            }
            float ms = 0.f;
            if (q == hipSuccess && hipEventElapsedTime(&ms, t.start[i], t.stop[i]) == hipSuccess)
                t.ns_per_update[i] = (double)ms * 1e6 / t.in_flight[i];
            else
                t.ns_per_update[i] = 1e30;  // not usable: ranks last
            t.in_flight[i] = 0;
        }
        all = all && t.ns_per_update[i] >= 0;
    }
    if (all && t.best < 0) {
        t.best = 0;
        for (size_t i = 1; i < t.ns_per_update.size(); ++i)
            if (t.ns_per_update[i] < t.ns_per_update[(size_t)t.best]) t.best = (int)i;
    }
}

}  // namespace

// Returns the block size to use (0 = default) and, while the shape is being
// tuned, events to record around the launch plus a slot for
// batch_threads_done.  No call waits: each of the first calls for a new
// shape times one candidate that has not been timed yet, and the timings
// are read by later calls once their launches have completed.
int batch_threads_for(int max_L, int count, bool word, hipStream_t stream, hipEvent_t *start, hipEvent_t *stop,
                      int *slot)
{
    (void)stream;
    *start = *stop = nullptr;
    *slot = -1;
    if (const int pinned = pinned_batch_threads()) return pinned;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const TuneKey key = tune_key(max_L, count, word);
    TuneEntry &t = g_tune[key];
    if (t.candidates.empty()) {
        if (word) {
            // at most 8 threads per a-word are used
            const int words = max_L * max_L / 128;
            for (int c : {1024, 512, 256, 128})
                if (c <= std::max(128, 8 * words) && (c >= 256 || words <= 128)) t.candidates.push_back(c);
        } else {
            const int calls = max_L * max_L / 16;
            for (int c : {1024, 512, 256})
                if (c / 2 < calls || c == 256) t.candidates.push_back(c);
        }
        const size_t n = t.candidates.size();
        t.ns_per_update.assign(n, -1.0);
        t.in_flight.assign(n, 0.0);
        t.start.assign(n, nullptr);
        t.stop.assign(n, nullptr);
    }
    harvest(t);
    if (t.best >= 0) return t.candidates[(size_t)t.best];
    for (size_t i = 0; i < t.candidates.size(); ++i) {
        if (t.ns_per_update[i] < 0 && t.in_flight[i] == 0) {
            if (!t.start[i]) {
                if (hipEventCreate(&t.start[i]) != hipSuccess) return 0;
                if (hipEventCreate(&t.stop[i]) != hipSuccess) {
                    (void)hipEventDestroy(t.start[i]);
                    t.start[i] = nullptr;
                    return 0;
                }
            }
            *start = t.start[i];
            *stop = t.stop[i];
            t.in_flight[i] = -1.0;  // no other call takes these events meanwhile
            const auto entry = std::make_pair(key, (int)i);
            auto it = std::find(g_tune_slots.begin(), g_tune_slots.end(), entry);
            if (it == g_tune_slots.end()) it = g_tune_slots.insert(g_tune_slots.end(), entry);
            *slot = (int)(it - g_tune_slots.begin());
            return t.candidates[i];
        }
    }
    return 0;  // every untimed candidate has a launch in flight: the default meanwhile
}

// The launch timed for `slot` has been enqueued between its events with
// `site_updates` site updates; its time is read by a later call.
void batch_threads_done(int slot, double site_updates)
{
    if (slot < 0) return;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto &entry = g_tune_slots[(size_t)slot];
    TuneEntry &t = g_tune[entry.first];
    t.in_flight[(size_t)entry.second] = site_updates > 0 ? site_updates : 1.0;
}

// The tuned block size for a batch shape if tuning has finished (reading
// completed timings first), else 0 (the default); never launches anything.
int batch_threads_tuned(int max_L, int count, bool word)
{
    if (const int pinned = pinned_batch_threads()) return pinned;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(tune_key(max_L, count, word));
    if (it == g_tune.end()) return 0;
    harvest(it->second);
    return it->second.best >= 0 ? it->second.candidates[(size_t)it->second.best] : 0;
}

int enqueue_observables_batch(lattice *const *hs, int32_t count, unsigned long long *dev, hipStream_t stream)
{
    for (int32_t b = 0; b < count; b += kMaxBatch) {
        BatchArgs a{};
        a.count = std::min<int32_t>(kMaxBatch, count - b);
        for (int i = 0; i < a.count; ++i) a.scratch[i] = hs[b + i]->d_scratch;
        const hipError_t e = launch_observables_batch(a, dev + 10 * (size_t)b, stream);
        if (e != hipSuccess) return hip_fail(e, "batched observables launch");
    }
    return LAT_OK;
}

// Batched path: lattices resident in LDS, up to kMaxBatch per launch.
int enqueue_lds_sweeps(lattice *const *hs, int32_t count, const uint32_t *sweeps, uint32_t uniform,
                       hipStream_t stream, bool tune, unsigned long long *obs_dev)
{
    // LATTICE_LDS_SITE=1 keeps every batch on the per-site form (tests compare the two)
    const char *env = std::getenv("LATTICE_LDS_SITE");
    const bool force_site = env && env[0] == '1';
    for (int32_t b = 0; b < count; b += kMaxBatch) {
        BatchArgs a{};
        a.count = std::min<int32_t>(kMaxBatch, count - b);
        int max_L = 0;
        double updates = 0;
        bool word = !force_site;
        for (int i = 0; i < a.count; ++i) {
            a.scratch[i] = hs[b + i]->d_scratch;
            a.sweeps[i] = sweeps ? sweeps[b + i] : uniform;
            max_L = std::max(max_L, hs[b + i]->L);
            updates += (double)hs[b + i]->N * a.sweeps[i];
            word = word && hs[b + i]->L % 64 == 0;
        }
        hipEvent_t t0 = nullptr, t1 = nullptr;
        int slot = -1;
        const int threads = tune ? batch_threads_for(max_L, a.count, word, stream, &t0, &t1, &slot)
                                 : batch_threads_tuned(max_L, a.count, word);
        a.obs_out = obs_dev ? obs_dev + 10 * (size_t)b : nullptr;
        if (t0) (void)hipEventRecord(t0, stream);
        hipError_t e = launch_sweep_lds(a, max_L, threads, word, stream);
        if (e != hipSuccess) return hip_fail(e, "batched kernel launch");
        if (t1) {
            (void)hipEventRecord(t1, stream);
            batch_threads_done(slot, updates);
        }
        for (int i = 0; i < a.count; ++i) hs[b + i]->done += a.sweeps[i];
    }
    return LAT_OK;
}

// v = (tracker nD, nV, nJ, sum S, sum S^2, bonds SS, bonds ss, M, M_st, C_st).
bool barrier_may_time_out(const lattice *h)
{
    return h->ran_persistent || (h->path == kPathPhase && h->tuning.persistent);
}

void fill_obs(const lattice *h, const int64_t *v, lat_obs *out)
{
    out->sweep = h->done;
    out->track_nD = v[0];
    out->track_nV = v[1];
    out->track_nJ = v[2];
    out->sum_S = v[3];
    out->n_charged = v[4];
    out->bond_SS = v[5];
    out->bond_ss = v[6];
    out->M = v[7];
    out->M_stag = v[8];
    out->C_stag = v[9];
    out->E = h->Delta * (double)out->n_charged + h->V * (double)out->bond_SS + 0.25 * h->J * (double)out->bond_ss;
}

// Parameter checks shared by lattice_create and the server's submit:
// geometry, finite couplings, T > 0, and the charge target of eq. (2) (from
// the given codes, which must lie in 0..3, or from n and n_charged).
int validate_params(const lat_params *p, int64_t *Q_out, int64_t *Nc_out)
{
    if (!valid_geometry(p->L, p->encoding))
        return fail(LAT_EINVAL, "invalid L for the encoding (int8: L%4==0; 2-bit: L%64==0; 4 <= L <= 32768)");
    if (!std::isfinite(p->Delta) || !std::isfinite(p->V) || !std::isfinite(p->J) || !std::isfinite(p->T) ||
        !std::isfinite(p->n))
        return fail(LAT_EINVAL, "parameters must be finite");
    if (!(p->T > 0.0)) return fail(LAT_EINVAL, "T must be > 0");
    int64_t Q = 0, Nc = 0;
    if (p->init_codes) {
        const int64_t N = (int64_t)p->L * p->L;
        for (int64_t i = 0; i < N; ++i) {
            const int c = p->init_codes[i];
            if (c < 0 || c > 3) return fail(LAT_EINVAL, "init code outside 0..3");
            Q += c == 2 ? 1 : (c == 3 ? -1 : 0);
            Nc += c >= 2;
        }
    } else {
        const int rc = charge_target(p->L, p->n, p->n_charged, &Q, &Nc);
        if (rc) return rc;
    }
    *Q_out = Q;
    *Nc_out = Nc;
    return LAT_OK;
}

}  // namespace detail
}  // namespace lat

namespace {

int enqueue_sweeps(lattice *h, uint32_t sweeps, hipStream_t stream)
{
    if (sweeps == 0) return LAT_OK;
    lattice *one[1] = {h};
    // the multi-block path takes the persistent launch where it can run
    if (h->path != kPathLds) return enqueue_offchip_sweeps(one, 1, nullptr, sweeps, stream);
    // a lone lattice is not autotuned (tuning synchronises); it takes the
    // block size tuned for its shape by an earlier batch, else the default
    return enqueue_lds_sweeps(one, 1, nullptr, sweeps, stream, /*tune=*/false);
}

// Sweep path of a new lattice.  Default: the one-block LDS kernel up to
// kLdsRouteMaxL, whose single compute unit is then still faster than a
// multi-block launch series; the multi-block word kernel up to kWordsMaxL;
// the one-thread-per-word phase kernel above.  LATTICE_PATH=lds|words|phase
// forces a path where it applies (tests run every path at small sizes);
// LATTICE_FORCE_PHASE_KERNELS=1 is the same as LATTICE_PATH=phase.
constexpr int kLdsRouteMaxL = 256;
constexpr int kWordsMaxL = 2048;

int choose_path(int L, int enc)
{
    const bool words_ok = L % 64 == 0 && L <= kWordsMaxL;
    if (const char *v = std::getenv("LATTICE_PATH")) {
        const std::string want(v);
        if (want == "lds" && L <= kLdsMaxL) return kPathLds;
        if (want == "words" && words_ok) return kPathWords;
        if (want == "phase") return kPathPhase;
    }
    if (const char *force = std::getenv("LATTICE_FORCE_PHASE_KERNELS"))
        if (std::atoi(force) != 0) return kPathPhase;
    (void)enc;
    if (L <= (L % 64 == 0 ? kLdsRouteMaxL : kLdsMaxL)) return kPathLds;
    return words_ok ? kPathWords : kPathPhase;
}

}  // namespace

extern "C" {

size_t lattice_state_bytes(int32_t L, int32_t encoding)
{
    if (!valid_geometry(L, encoding)) return 0;
    const size_t N = (size_t)L * L;
    return encoding == LAT_ENC_INT8 ? N : N / 4;
}

size_t lattice_scratch_bytes(int32_t L, int32_t encoding)
{
    if (!valid_geometry(L, encoding)) return kScrBytes;
    return kScrBytes + (int8_packs(L, encoding) ? (size_t)L * L / 4 : 0);
}

int lattice_charge_target(int32_t L, double n, int64_t n_charged, int64_t *Q, int64_t *Nc)
{
    return guarded("lattice_charge_target", [&]() -> int {
        if (!Q || !Nc) return fail(LAT_EINVAL, "null output pointer");
        if (L < 1 || L > kMaxL) return fail(LAT_EINVAL, "L out of range");
        return charge_target(L, n, n_charged, Q, Nc);
    });
}

int lattice_create(const lat_params *p, void *d_state, size_t state_bytes, void *d_scratch, size_t scratch_bytes,
                   void *hip_stream, lattice **out)
{
    return guarded("lattice_create", [&]() -> int {
        g_err.clear();
        if (!p || !out) return fail(LAT_EINVAL, "null params or output handle");
        *out = nullptr;
        int64_t Q = 0, Nc = 0;
        int rc = validate_params(p, &Q, &Nc);
        if (rc) return rc;
        if (!d_state || !d_scratch) return fail(LAT_EINVAL, "null device buffer");
        if (state_bytes < lattice_state_bytes(p->L, p->encoding)) return fail(LAT_ENOMEM, "state buffer too small");
        if (scratch_bytes < lattice_scratch_bytes(p->L, p->encoding)) return fail(LAT_ENOMEM, "scratch buffer too small");

        const int64_t N = (int64_t)p->L * p->L;
        std::vector<int8_t> codes;
        if (p->init_codes)
            codes.assign(p->init_codes, p->init_codes + N);
        else
            seeded_init(p->L, p->seed, (Nc + Q) / 2, (Nc - Q) / 2, codes);
        std::vector<uint8_t> dev;
        to_device_layout(p->L, p->encoding, codes, dev);
        std::vector<uint32_t> tab, dev_tab, trans, trans_d;
        build_threshold_table(p->Delta, p->V, p->J, p->T, tab);
        build_device_table(tab, dev_tab);
        build_transition_table(trans, trans_d);
        {
            static std::once_flag once;
            static hipError_t init_err = hipSuccess;
            std::call_once(once, [] {
                init_err = init_kernel_attributes();
                if (init_err == hipSuccess) init_err = init_map_kernel_attributes();
            });
            if (init_err != hipSuccess) return hip_fail(init_err, "kernel set-up");
        }

        lattice *h = new lattice();
        h->L = p->L;
        h->enc = p->encoding;
        h->N = N;
        h->Q = Q;
        h->Nc = Nc;
        h->n = p->n;
        h->Delta = p->Delta;
        h->V = p->V;
        h->J = p->J;
        h->T = p->T;
        h->seed = p->seed;
        h->start_sweep = p->start_sweep;
        h->d_state = d_state;
        h->d_scratch = (uint8_t *)d_scratch;
        h->stream = (hipStream_t)hip_stream;
        h->tuning = tuning_from_env();
        h->path = choose_path(p->L, p->encoding);
        h->packed = h->path != kPathLds && int8_packs(p->L, p->encoding);
        h->magic = kMagic;
        LatDesc desc{};
        desc.state = d_state;
        desc.L = p->L;
        desc.enc = p->encoding;
        desc.key0 = (uint32_t)p->seed;
        desc.key1 = (uint32_t)(p->seed >> 32);
        desc.next_sweep = p->start_sweep;

        hipError_t e = hipMemcpyAsync(d_state, dev.data(), dev.size(), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->d_scratch + kScrDevTab, dev_tab.data(), dev_tab.size() * 4, hipMemcpyHostToDevice,
                               h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->d_scratch + kScrTrans, trans.data(), trans.size() * 4, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->d_scratch + kScrTransD, trans_d.data(), trans_d.size() * 4, hipMemcpyHostToDevice,
                               h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->d_scratch + kScrFullTab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->d_scratch + kScrDesc, &desc, sizeof(desc), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = launch_zero_i64((unsigned long long *)(h->d_scratch + kScrTrack), 11, h->stream);
        if (e == hipSuccess) e = launch_zero_i64((unsigned long long *)(h->d_scratch + kScrTrackBase), 3, h->stream);
        if (e == hipSuccess) e = launch_zero_i64((unsigned long long *)(h->d_scratch + kScrSlots), 3 * kMaxSlots, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // host staging buffers die with this frame
        if (e != hipSuccess) {
            h->magic = 0;
            delete h;
            return hip_fail(e, "lattice_create");
        }
        *out = h;
        return LAT_OK;
    });
}

int lattice_sweep(lattice *h, uint32_t sweeps)
{
    return guarded("lattice_sweep", [&]() -> int {
        if (!live(h)) return fail(LAT_ESTATE, "null or destroyed handle");
        return enqueue_sweeps(h, sweeps, h->stream);
    });
}

int lattice_sweep_batch(lattice *const *hs, int32_t count, uint32_t sweeps, void *hip_stream)
{
    return guarded("lattice_sweep_batch", [&]() -> int {
        if (count < 0 || (count > 0 && !hs)) return fail(LAT_EINVAL, "bad batch");
        for (int32_t i = 0; i < count; ++i)
            if (!live(hs[i])) return fail(LAT_ESTATE, "null or destroyed handle in batch");
        {
            std::vector<const lattice *> seen(hs, hs + count);
            std::sort(seen.begin(), seen.end());
            if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
                return fail(LAT_EINVAL, "a lattice appears twice in the batch");
        }
        if (sweeps == 0) return LAT_OK;
        std::vector<lattice *> small, big;
        for (int32_t i = 0; i < count; ++i) (hs[i]->path == kPathLds ? small : big).push_back(hs[i]);
        int rc = enqueue_lds_sweeps(small.data(), (int32_t)small.size(), nullptr, sweeps, (hipStream_t)hip_stream);
        if (rc == LAT_OK && !big.empty())
            rc = enqueue_offchip_sweeps(big.data(), (int32_t)big.size(), nullptr, sweeps, (hipStream_t)hip_stream);
        return rc;
    });
}

int lattice_observables_batch(lattice *const *hs, int32_t count, void *d_out, size_t out_bytes, lat_obs *out,
                              void *hip_stream)
{
    return guarded("lattice_observables_batch", [&]() -> int {
        if (count < 0 || (count > 0 && (!hs || !out || !d_out))) return fail(LAT_EINVAL, "bad batch");
        if (out_bytes < (size_t)count * 80u) return fail(LAT_ENOMEM, "output buffer smaller than 80 bytes per lattice");
        for (int32_t i = 0; i < count; ++i)
            if (!live(hs[i])) return fail(LAT_ESTATE, "null or destroyed handle in batch");
        hipStream_t stream = (hipStream_t)hip_stream;
        const int rc = enqueue_observables_batch(hs, count, (unsigned long long *)d_out, stream);
        if (rc) return rc;
        std::vector<int64_t> v((size_t)count * 10);
        hipError_t e = hipSuccess;
        if (count > 0) e = hipMemcpyAsync(v.data(), d_out, v.size() * 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        // lattices swept by the persistent kernel: its bounded device-wide
        // barrier flags a time-out in the lattice's error word
        for (int32_t i = 0; i < count && e == hipSuccess; ++i) {
            if (!barrier_may_time_out(hs[i])) continue;
            uint32_t err = 0;
            e = hipMemcpy(&err, hs[i]->d_scratch + kScrErr, sizeof(err), hipMemcpyDeviceToHost);
            if (e == hipSuccess && (err & 1u))
                return fail(LAT_EHIP, "a device-wide phase barrier timed out; the state is invalid");
        }
        if (e != hipSuccess) return hip_fail(e, "lattice_observables_batch");
        for (int32_t i = 0; i < count; ++i) fill_obs(hs[i], &v[10 * (size_t)i], &out[i]);
        return LAT_OK;
    });
}

int lattice_sweep_series(lattice *h, uint32_t intervals, uint32_t every, void *d_series, size_t series_bytes)
{
    return guarded("lattice_sweep_series", [&]() -> int {
        if (!live(h)) return fail(LAT_ESTATE, "null or destroyed handle");
        if (every == 0 || (intervals > 0 && !d_series)) return fail(LAT_EINVAL, "every must be > 0 and d_series set");
        if (series_bytes / kSeriesRecord < intervals)
            return fail(LAT_ENOMEM, "series buffer smaller than 88 bytes per interval");
        if (intervals == 0) return LAT_OK;
        lattice *one[1] = {h};
        hipStream_t st = h->stream;
        uint32_t *work = (uint32_t *)(h->d_scratch + kScrWork);
        // a packed int8 lattice stays on its 2-bit copy for the whole series
        if (h->packed) {
            const hipError_t e = launch_pack_int8((const int8_t *)h->d_state, work, h->L, st);
            if (e != hipSuccess) return hip_fail(e, "int8 pack launch");
        }
        // the whole series in persistent launches where they can run
        bool ran = false;
        const int rc0 = enqueue_words_persistent(one, 1, nullptr, intervals, every, (long long *)d_series, st, &ran);
        if (rc0) return rc0;
        for (uint32_t k = 0; k < intervals && !ran; ++k) {
            const int rc = h->path == kPathLds ? enqueue_lds_sweeps(one, 1, nullptr, every, st, /*tune=*/false)
                                               : enqueue_offchip_sweeps(one, 1, nullptr, every, st, /*convert=*/false);
            if (rc) return rc;
            long long *rec = (long long *)((uint8_t *)d_series + kSeriesRecord * (size_t)k);
            const hipError_t e = launch_observables(h->d_scratch, h->packed ? (const void *)work : h->d_state, h->L,
                                                    h->packed ? LAT_ENC_2BIT : h->enc, st, rec);
            if (e != hipSuccess) return hip_fail(e, "observables launch");
        }
        if (h->packed) {
            const hipError_t e = launch_unpack_int8(work, (int8_t *)h->d_state, h->L, st);
            if (e != hipSuccess) return hip_fail(e, "int8 unpack launch");
        }
        return LAT_OK;
    });
}

int lattice_series_read(lattice *h, const void *d_series, uint32_t intervals, lat_obs *out)
{
    return guarded("lattice_series_read", [&]() -> int {
        if (!live(h)) return fail(LAT_ESTATE, "null or destroyed handle");
        if (intervals > 0 && (!d_series || !out)) return fail(LAT_EINVAL, "null series or output");
        if (intervals == 0) return LAT_OK;
        std::vector<int64_t> v((size_t)intervals * (kSeriesRecord / 8));
        uint32_t err = 0;
        hipError_t e = hipMemcpyAsync(v.data(), d_series, v.size() * 8, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&err, h->d_scratch + kScrErr, sizeof(err), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "lattice_series_read");
        if (err & 1u) return fail(LAT_EHIP, "a device-wide phase barrier timed out; the state is invalid");
        for (uint32_t k = 0; k < intervals; ++k) {
            const int64_t *rec = &v[(kSeriesRecord / 8) * (size_t)k];
            fill_obs(h, rec, &out[k]);
            out[k].sweep = (uint64_t)rec[10] - h->start_sweep;
        }
        return LAT_OK;
    });
}

int lattice_observables(lattice *h, lat_obs *out)
{
    return guarded("lattice_observables", [&]() -> int {
        if (!live(h)) return fail(LAT_ESTATE, "null or destroyed handle");
        if (!out) return fail(LAT_EINVAL, "null output");
        unsigned long long *track = (unsigned long long *)(h->d_scratch + kScrTrack);
        hipError_t e = launch_observables(h->d_scratch, h->d_state, h->L, h->enc, h->stream);
        int64_t v[11];  // tracker, 7 sums, error flags
        if (e == hipSuccess) e = hipMemcpyAsync(v, track, sizeof(v), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "lattice_observables");
        if ((uint32_t)v[10] & 1u) return fail(LAT_EHIP, "a device-wide phase barrier timed out; the state is invalid");
        fill_obs(h, v, out);
        return LAT_OK;
    });
}

int lattice_read_state(lattice *h, int8_t *host_codes)
{
    return guarded("lattice_read_state", [&]() -> int {
        if (!live(h)) return fail(LAT_ESTATE, "null or destroyed handle");
        if (!host_codes) return fail(LAT_EINVAL, "null output");
        std::vector<uint8_t> dev(lattice_state_bytes(h->L, h->enc));
        hipError_t e = hipMemcpyAsync(dev.data(), h->d_state, dev.size(), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "lattice_read_state");
        from_device_layout(h->L, h->enc, dev, host_codes);
        return LAT_OK;
    });
}

int lattice_destroy(lattice *h)
{
    return guarded("lattice_destroy", [&]() -> int {
        if (!live(h)) return fail(LAT_ESTATE, "null or destroyed handle");
        h->magic = 0;
        delete h;
        return LAT_OK;
    });
}

const char *lattice_last_error(void) { return g_err_fixed ? g_err_fixed : g_err.c_str(); }

}  // extern "C"
