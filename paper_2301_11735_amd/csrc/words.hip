// gfx950 multi-block phase kernels of the coupled-pair Metropolis sweep
// (arXiv:2301.11735, section 3.1 update, section 3.2 parallel form) for
// lattices of medium size, and the int8 <-> 2-bit class-layout conversion.
//
// A phase of a lattice with L = 512..2048 has only 2k..33k a-words: one
// thread per word (16 pairs each, as in the large-lattice phase kernel)
// leaves most of the chip idle and puts 16 dependent pair steps on the
// critical path.  Here Q lanes share a word (word_task.h), a lattice spreads
// over many 256-thread blocks, and one launch can hold several lattices
// (the server's large requests), each at its own sweep.  The schedule of a
// sweep is computed on the device from the lattice's seed and sweep index,
// so a series of launches does not depend on host state and can be
// replayed from a HIP graph.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device_common.h"
#include "word_task.h"

namespace lat {
namespace {

template <int Q>
__global__ void __launch_bounds__(kWordsPhaseMaxThreads) k_phase_words(WordsArgs a)
{
    __shared__ uint2 s_tab[kDevTabEntries];
    __shared__ uint4 s_transd[kTransEntries];
    // the lattice of this block (uniform; at most kWordsBatch lattices)
    int li = 0;
    while (li + 1 < a.count && blockIdx.x >= a.first_block[li + 1]) ++li;
    if (a.iter >= a.sweeps[li]) return;  // the whole block: no barrier is skipped by part of it
    uint8_t *scr = a.scratch[li];
    const LatDesc d = *(const LatDesc *)(scr + kScrDesc);
    uint32_t *st = d.enc == 1 ? (uint32_t *)d.state : (uint32_t *)(scr + kScrWork);
    {
        const uint2 *g_tab = (const uint2 *)(scr + kScrDevTab);
        const uint4 *g_transd = (const uint4 *)(scr + kScrTransD);
        for (int i = threadIdx.x; i < kDevTabEntries; i += blockDim.x) s_tab[i] = g_tab[i];
        for (int i = threadIdx.x; i < kTransEntries; i += blockDim.x) s_transd[i] = g_transd[i];
    }
    const uint64_t s = d.next_sweep + a.iter;
    int r, mm[4], kk[4];
    device_schedule(d.L, d.key0, d.key1, s, r, mm, kk);
    WordPhase f;
    word_phase_setup(f, d.L, d.key0, d.key1, s, a.p, r, mm, kk);
    const uint32_t csz = (uint32_t)f.H * (uint32_t)f.W;
    __syncthreads();

    const uint32_t b = blockIdx.x - a.first_block[li];
    const uint32_t task = b * blockDim.x + threadIdx.x;
    int tr[3] = {0, 0, 0};
    // tasks = Q * csz is a multiple of Q, so a word's lanes are all in or all out
    if (task < (uint32_t)Q * csz) word_task<Q, false, kDrawInPlace, true>(st, f, task, s_tab, s_transd, tr);
    block_reduce_add<3>(tr, (unsigned long long *)(scr + kScrSlots) + 3 * (size_t)b);
}

// Adds the block's sums of m (per thread: tracker moves 0-2, spin,
// staggered spin and staggered charge moves 3-5) to an observation record
// (tracker 0-2, sums 3-9): m[0..2] to fields 0-2 and 4-6, m[3..5] to 7-9.
__device__ __forceinline__ void add_record_moves(long long (&m)[6], unsigned long long *rec)
{
    __shared__ long long part[16][6];
    wave_partials<6, long long>(m, part);
    __syncthreads();
    if (threadIdx.x < 9) {
        const int i = threadIdx.x < 6 ? (int)threadIdx.x % 3 : (int)threadIdx.x - 3;
        const int field = threadIdx.x < 3 ? (int)threadIdx.x : (int)threadIdx.x + 1;
        const int nw = (int)(blockDim.x >> 6);
        long long sum = 0;
        for (int w = 0; w < nw; ++w) sum += part[w][i];
        if (sum != 0) atomicAdd(&rec[field], (unsigned long long)sum);
    }
    __syncthreads();  // part is reused at the next interval
}

// Persistent form: the sweeps of a whole call of up to kWordsBatch lattices,
// or a whole observation series of one lattice, in one launch of
// co-resident blocks (cooperative launch); blocks first_block[i] ..
// first_block[i+1]-1 update lattice i.  Tables are staged once; every phase
// is one grid-stride pass over each lattice's a-word tasks by its own blocks,
// followed by a device-wide barrier of all blocks.  Sweep it of the launch
// (interval k, sweep e of it: it = k every + e) is sweep next_sweep + it of
// every lattice with sweeps[i] > it; the blocks of the others only meet the
// barriers.  All lattice words are read and written at device coherence, so
// the barrier needs no cache write-back or invalidation (measured on MI355X
// with 128 blocks: 2.3 us a barrier, against 6.9 us with one release/acquire
// fence pair per block and 12-14 us with a fence pair in every wave).
//
// Obs (a series with records, one lattice): the records start as the
// lattice's state before the launch (k_series_init: tracker total and the
// seven sums), and at the end of interval k every block adds its moves since
// the launch began to record k: its tracker sums (to the tracker and to the
// charged-site count and the two bond sums, which change by exactly them)
// and the spin, staggered spin and staggered charge moves of the words it
// wrote.  The lattice is not read for the records, so no barrier beyond the
// phases' is needed; the records are whole when the launch ends.
template <int Q, bool Obs>
__global__ void __launch_bounds__(kWordsThreads) k_words_series(WordsSeriesArgs a)
{
    __shared__ uint2 s_tab[kDevTabEntries];
    __shared__ uint4 s_transd[kTransEntries];
    int li = 0;  // this block's lattice (uniform)
    while (li + 1 < a.count && blockIdx.x >= a.first_block[li + 1]) ++li;
    uint8_t *scr = a.scratch[li];
    const LatDesc d = *(const LatDesc *)(scr + kScrDesc);
    uint32_t *st = d.enc == 1 ? (uint32_t *)d.state : (uint32_t *)(scr + kScrWork);
    {
        const uint2 *g_tab = (const uint2 *)(scr + kScrDevTab);
        const uint4 *g_transd = (const uint4 *)(scr + kScrTransD);
        for (int i = threadIdx.x; i < kDevTabEntries; i += blockDim.x) s_tab[i] = g_tab[i];
        for (int i = threadIdx.x; i < kTransEntries; i += blockDim.x) s_transd[i] = g_transd[i];
    }
    __syncthreads();
    unsigned *counter = (unsigned *)(a.scratch[0] + kScrBarrier), *err = (unsigned *)(scr + kScrErr);
    const uint32_t b = blockIdx.x - a.first_block[li], nb = a.first_block[li + 1] - a.first_block[li];
    const uint32_t my_sweeps = a.sweeps[li];
    const uint32_t csz = (uint32_t)(d.L >> 1) * (uint32_t)(d.L >> 6);
    const uint32_t n_tasks = (uint32_t)Q * csz, stride = nb * blockDim.x;
    const uint32_t first = b * blockDim.x + threadIdx.x;
    // At most one task a thread (uniform per lattice): its Philox draws for
    // the next phase are made while the block waits at the barrier, where
    // they depend on nothing the other blocks write.
    const bool one = stride >= n_tasks, mine = one && first < n_tasks;
    const int q = (int)(first & (uint32_t)(Q - 1));
    u32x4 pre[kTaskCalls<Q>];
    uint32_t c0 = 0;
    auto draws = [&](uint64_t s, int p) {
#pragma unroll
        for (int i = 0; i < kTaskCalls<Q>; ++i)
            pre[i] = philox4x32_10((uint32_t)s, (uint32_t)p, c0 + (uint32_t)call_of_task<Q>(q, i), (uint32_t)(s >> 32),
                                   d.key0, d.key1);
    };
    int r, mm[4], kk[4];
    device_schedule(d.L, d.key0, d.key1, d.next_sweep, r, mm, kk);
    if (mine && my_sweeps > 0) {
        WordPhase f0;
        word_phase_setup(f0, d.L, d.key0, d.key1, d.next_sweep, 0, r, mm, kk);
        c0 = task_call0<Q>(f0, first);
        draws(d.next_sweep, 0);
    }
    int tr[3] = {0, 0, 0};
    int dv[3] = {0, 0, 0};  // Obs: spin, staggered spin, staggered charge moves
    unsigned arrivals = 0;
    for (uint32_t k = 0; k < a.intervals; ++k) {
        for (uint32_t e = 0; e < a.every; ++e) {
            const uint32_t it = k * a.every + e;
            const uint64_t s = d.next_sweep + it;
            for (int p = 0; p < 4; ++p) {
                if (it < my_sweeps) {
                    WordPhase f;
                    word_phase_setup(f, d.L, d.key0, d.key1, s, p, r, mm, kk);
                    if (one) {
                        if (mine)
                            word_task<Q, false, kDrawGiven, true, true, Obs>(st, f, first, s_tab, s_transd, tr, pre, 0,
                                                                             0, dv);
                    } else {
                        // stride is a multiple of Q: a word's lanes are all in or all out
                        for (uint32_t t = first; t < n_tasks; t += stride)
                            word_task<Q, false, kDrawInPlace, true, true, Obs>(st, f, t, s_tab, s_transd, tr, nullptr,
                                                                               0, 0, dv);
                    }
                }
                if constexpr (Obs) {
                    if (p == 3 && e + 1 == a.every) {
                        unsigned long long *rec =
                            (unsigned long long *)(a.records + (kSeriesRecord / 8) * (size_t)k);
                        long long m[6] = {tr[0], tr[1], tr[2], dv[0], dv[1], dv[2]};
                        add_record_moves(m, rec);
                        if (b == 0 && threadIdx.x == 0)
                            rec[10] = (unsigned long long)(d.next_sweep + (uint64_t)(k + 1) * a.every);
                    }
                }
                arrivals += gridDim.x;
                grid_arrive_coherent(counter);
                // the next phase's schedule and draws, while the others arrive
                const uint32_t it_next = p < 3 ? it : it + 1;
                const uint64_t s_next = p < 3 ? s : s + 1;
                if (p == 3) device_schedule(d.L, d.key0, d.key1, s_next, r, mm, kk);
                if (mine && it_next < my_sweeps) draws(s_next, p < 3 ? p + 1 : 0);
                grid_wait_coherent(counter, arrivals, err, a.barrier_ticks);
            }
        }
    }
    block_reduce_add<3>(tr, (unsigned long long *)(scr + kScrSlots) + 3 * (size_t)b);
    // every block read the descriptor before its first barrier
    if (b == 0 && threadIdx.x == 0 && arrivals > 0)
        ((LatDesc *)(scr + kScrDesc))->next_sweep = d.next_sweep + my_sweeps;
}

// Records of a series before it runs: the tracker total so far (slots and
// base) and the seven observable sums of the lattice's current state (its
// 2-bit copy for an int8 lattice), in every record.  One block.
__global__ void __launch_bounds__(1024) k_series_init(const uint8_t *scr, long long *records, uint32_t intervals)
{
    const LatDesc d = *(const LatDesc *)(scr + kScrDesc);
    const uint32_t *st = d.enc == 1 ? (const uint32_t *)d.state : (const uint32_t *)(scr + kScrWork);
    long long t3[3] = {0, 0, 0};
    const long long *slots = (const long long *)(scr + kScrSlots);
    for (int i = threadIdx.x; i < kMaxSlots; i += blockDim.x) {
        t3[0] += slots[3 * i];
        t3[1] += slots[3 * i + 1];
        t3[2] += slots[3 * i + 2];
    }
    if (threadIdx.x == 0) {
        const long long *base = (const long long *)(scr + kScrTrackBase);
        t3[0] += base[0];
        t3[1] += base[1];
        t3[2] += base[2];
    }
    long long v[7] = {0, 0, 0, 0, 0, 0, 0};
    const uint32_t n = 8u * (uint32_t)(d.L >> 1) * (uint32_t)(d.L >> 6);
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) obs_word_2bit(st, d.L, i, v);
    __shared__ long long tot[10];
    block_reduce_store<3>(t3, tot);
    block_reduce_store<7>(v, tot + 3);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < intervals; k += blockDim.x) {
        long long *rec = records + (kSeriesRecord / 8) * (size_t)k;
        for (int q = 0; q < 10; ++q) rec[q] = tot[q];
        rec[10] = 0;
    }
}

__global__ void k_advance_words(WordsArgs a)
{
    if (blockIdx.x == 0 && (int)threadIdx.x < a.count)
        ((LatDesc *)(a.scratch[threadIdx.x] + kScrDesc))->next_sweep += a.sweeps[threadIdx.x];
}

// Thread (y, j): the 64 int8 codes of row y starting at x = 64j, i.e. word j
// of class row y/2 of the four classes 4(y mod 2) + cx (site x = 4X + cx,
// X = 16j + t at bits 2t).  Byte cx of 32-bit word t of the 64 codes is
// site 4(16j + t) + cx.
__global__ void __launch_bounds__(256) k_pack_int8(const int8_t *__restrict__ src, uint32_t *__restrict__ dst,
                                                   int L)
{
    const uint32_t W = (uint32_t)L >> 6, H = (uint32_t)L >> 1, csz = H * W;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)L * W) return;
    const uint32_t y = i / W, j = i - y * W;
    const uint4 *row = (const uint4 *)(src + (size_t)y * L + 64u * j);
    uint32_t w[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint4 v = row[k];
        w[4 * k] = v.x;
        w[4 * k + 1] = v.y;
        w[4 * k + 2] = v.z;
        w[4 * k + 3] = v.w;
    }
    const uint32_t c0 = 4u * (y & 1u), Y = y >> 1;
#pragma unroll
    for (uint32_t cx = 0; cx < 4; ++cx) {
        uint32_t cw = 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) cw |= ((w[t] >> (8u * cx)) & 3u) << (2 * t);
        dst[(c0 + cx) * csz + Y * W + j] = cw;
    }
}

__global__ void __launch_bounds__(256) k_unpack_int8(const uint32_t *__restrict__ src, int8_t *__restrict__ dst,
                                                     int L)
{
    const uint32_t W = (uint32_t)L >> 6, H = (uint32_t)L >> 1, csz = H * W;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)L * W) return;
    const uint32_t y = i / W, j = i - y * W;
    const uint32_t c0 = 4u * (y & 1u), Y = y >> 1;
    uint32_t cw[4];
#pragma unroll
    for (uint32_t cx = 0; cx < 4; ++cx) cw[cx] = src[(c0 + cx) * csz + Y * W + j];
    uint4 *row = (uint4 *)(dst + (size_t)y * L + 64u * j);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = 4 * k + u;
            v[u] = ((cw[0] >> (2 * t)) & 3u) | (((cw[1] >> (2 * t)) & 3u) << 8) | (((cw[2] >> (2 * t)) & 3u) << 16) |
                   (((cw[3] >> (2 * t)) & 3u) << 24);
        }
        row[k] = make_uint4(v[0], v[1], v[2], v[3]);
    }
}

}  // namespace

// Lanes per a-word of the per-phase form.  Up to L = 1024: 4.  The form's
// main user below that size is the server's second stream, whose launches
// hold several lattices beside the on-chip kernel's blocks; there 4 lanes
// beat 8 (a 60 s served run: p99 0.224 s against 0.253-0.257 s, L = 512
// requests 0.246 against 0.277-0.280 s; 2 lanes: 0.232-0.236 s).
int words_lanes(int L)
{
    if (L <= 1024) return 4;
    if (L <= 2048) return 2;
    return 1;
}

hipError_t launch_phase_words(const WordsArgs &a, int Q, int threads, hipStream_t s)
{
    const dim3 grid(a.first_block[a.count]), block((unsigned)threads);
    switch (Q) {
    case 1: hipLaunchKernelGGL(k_phase_words<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_phase_words<2>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_phase_words<4>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(k_phase_words<8>, grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

namespace {
template <int Q>
const void *series_fn(bool obs)
{
    return obs ? (const void *)k_words_series<Q, true> : (const void *)k_words_series<Q, false>;
}
const void *series_fn_of(int Q, bool obs)
{
    switch (Q) {
    case 1: return series_fn<1>(obs);
    case 2: return series_fn<2>(obs);
    case 4: return series_fn<4>(obs);
    default: return series_fn<8>(obs);
    }
}
}  // namespace

int words_persistent_capacity(int Q, int threads)
{
    int dev = 0, coop = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 0;
    // the smaller of the two forms' (with and without records) resident blocks
    for (const bool obs : {false, true}) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, series_fn_of(Q, obs), threads, 0) != hipSuccess ||
            n < 1)
            return 0;
        per_cu = obs ? std::min(per_cu, n) : n;
    }
    return per_cu * cus;
}

hipError_t launch_words_series(const WordsSeriesArgs &a, int Q, hipStream_t s)
{
    // the launch's barrier counter lives in the first lattice's scratch
    hipError_t e = launch_zero_i64((unsigned long long *)(a.scratch[0] + kScrBarrier), 1, s);
    if (e != hipSuccess) return e;
    if (a.records) {
        hipLaunchKernelGGL(k_series_init, dim3(1), dim3(1024), 0, s, (const uint8_t *)a.scratch[0], a.records,
                           a.intervals);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    WordsSeriesArgs args = a;
    void *kargs[] = {&args};
    return hipLaunchCooperativeKernel(series_fn_of(Q, a.records != nullptr), dim3(a.first_block[a.count]),
                                      dim3((unsigned)a.threads), kargs, 0, s);
}

hipError_t launch_advance_words(const WordsArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance_words, dim3(1), dim3(kWordsBatch), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pack_int8(const int8_t *src, uint32_t *dst, int L, hipStream_t s)
{
    const uint32_t n = (uint32_t)L * ((uint32_t)L >> 6);
    hipLaunchKernelGGL(k_pack_int8, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, L);
    return hipGetLastError();
}

hipError_t launch_unpack_int8(const uint32_t *src, int8_t *dst, int L, hipStream_t s)
{
    const uint32_t n = (uint32_t)L * ((uint32_t)L >> 6);
    hipLaunchKernelGGL(k_unpack_int8, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, L);
    return hipGetLastError();
}

}  // namespace lat
