// gfx950 batched kernels (arXiv:2301.11735 section 3.2: several lattice
// copies processed together): one block per lattice, the lattice resident in
// LDS for all the sweeps of a launch, and the batched observable reduction.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device_common.h"
#include "word_task.h"

namespace lat {
namespace {

// ---------------------------------------------------------------------------
// Batched lattices (section 3.2: several lattice copies processed together),
// one block per lattice, the whole lattice resident in LDS for all sweeps of
// the launch.  LDS layout: the 8 sublattice classes, each (L/2) rows of
// Wp = ceil(L/64) words, site X of a class row at bits 2*(X&15) of word X>>4.
// Each thread owns Philox calls t = tid, tid + blockDim, ...: pairs 2t and
// 2t+1.  A pair's two sites are in words other pairs of the phase also own
// fields of, so the new codes are merged with LDS atomic xor; every read of
// an updated word extracts only the reader's own field, which nobody else
// writes, and neighbour words are never written in the phase.

struct LdsGeom {
    int L, Lq, H, Wp;
    uint32_t csz;  // words per class
    __device__ __forceinline__ uint32_t word(int c, int Y, int X) const
    {
        return (uint32_t)c * csz + (uint32_t)Y * Wp + (uint32_t)(X >> 4);
    }
};

__device__ __forceinline__ uint32_t lds_code(const uint32_t *lat, const LdsGeom &g, int c, int Y, int X)
{
    return (lat[g.word(c, Y, X)] >> (2 * (X & 15))) & 3u;
}

// Copy a lattice from its global state into the LDS class arrays (rows of
// Wp words, 16 sites per word; int8 states are packed on the way in), and back.
__device__ __forceinline__ void stage_lattice(uint32_t *lat, const LatDesc &d, const LdsGeom &g)
{
    const int L = g.L, Lq = g.Lq;
    const uint32_t nwords = 8u * g.csz;
    if (d.enc == 1) {
        const uint32_t *src = (const uint32_t *)d.state;  // same layout, Wp = L/64
        for (uint32_t i = threadIdx.x; i < nwords; i += blockDim.x) lat[i] = src[i];
    } else {
        const int8_t *src = (const int8_t *)d.state;
        for (uint32_t i = threadIdx.x; i < nwords; i += blockDim.x) {
            const int c = (int)(i / g.csz);
            const uint32_t rem = i - (uint32_t)c * g.csz;
            const int Y = (int)(rem / g.Wp), w = (int)(rem - (uint32_t)Y * g.Wp);
            const int x0 = c & 3, y = 2 * Y + (c >> 2);
            uint32_t v = 0;
            for (int t = 0; t < 16; ++t) {
                const int X = 16 * w + t;
                if (X < Lq) v |= ((uint32_t)src[(size_t)y * L + 4 * X + x0] & 3u) << (2 * t);
            }
            lat[i] = v;
        }
    }
}

__device__ __forceinline__ void unstage_lattice(const uint32_t *lat, const LatDesc &d, const LdsGeom &g)
{
    const int L = g.L;
    if (d.enc == 1) {
        uint32_t *dst = (uint32_t *)d.state;
        for (uint32_t i = threadIdx.x; i < 8u * g.csz; i += blockDim.x) dst[i] = lat[i];
    } else {
        int8_t *dst = (int8_t *)d.state;
        for (uint32_t i = threadIdx.x; i < (uint32_t)L * L; i += blockDim.x) {
            const int y = (int)(i / L), x = (int)(i - (uint32_t)y * L);
            dst[i] = (int8_t)lds_code(lat, g, 4 * (y & 1) + (x & 3), y >> 1, x >> 2);
        }
    }
}

__global__ void __launch_bounds__(1024) k_sweep_lds(BatchArgs args)
{
    __shared__ uint2 s_tab[kDevTabEntries];
    __shared__ uint2 s_trans[kTransEntries];
    extern __shared__ uint32_t lat[];
    uint8_t *scr = args.scratch[blockIdx.x];
    const LatDesc d = *(const LatDesc *)(scr + kScrDesc);
    stage_tables(s_tab, s_trans, (const uint2 *)(scr + kScrDevTab), (const uint2 *)(scr + kScrTrans));
    LdsGeom g;
    g.L = d.L;
    g.Lq = d.L >> 2;
    g.H = d.L >> 1;
    g.Wp = (g.Lq + 15) >> 4;
    g.csz = (uint32_t)g.H * g.Wp;
    const int L = g.L, Lq = g.Lq, H = g.H;

    stage_lattice(lat, d, g);
    __syncthreads();

    const uint32_t n_calls = (uint32_t)L * (uint32_t)L / 16u;
    int tr[3] = {0, 0, 0};
    const uint32_t my_sweeps = args.sweeps[blockIdx.x];
    for (uint64_t s = d.next_sweep; s < d.next_sweep + my_sweeps; ++s) {
        int r, mm[4], kk[4];
        device_schedule(L, d.key0, d.key1, s, r, mm, kk);
        for (int p = 0; p < 4; ++p) {
            const int pb = (p + r) & 3, carry = (p + r) >> 2;
            int dX = mm[p] + carry;
            if (dX >= Lq) dX -= Lq;
            const int cAL = p > 0 ? p - 1 : 3, cAR = p < 3 ? p + 1 : 0;
            const int cBL = pb > 0 ? 4 + pb - 1 : 7, cBR = pb < 3 ? 4 + pb + 1 : 4;
            for (uint32_t t = threadIdx.x; t < n_calls; t += blockDim.x) {
                const u32x4 w = philox4x32_10((uint32_t)s, (uint32_t)p, t, (uint32_t)(s >> 32), d.key0, d.key1);
                uint32_t packed = 0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t pi = 2u * t + (uint32_t)h;
                    const int Y = (int)(pi / (uint32_t)Lq), X = (int)pi - Y * Lq;
                    int Yb = Y + kk[p], Xb = X + dX;
                    if (Yb >= H) Yb -= H;
                    if (Xb >= Lq) Xb -= Lq;
                    const int Xl = X == 0 ? Lq - 1 : X - 1, Xr = X + 1 == Lq ? 0 : X + 1;
                    const int Xbl = Xb == 0 ? Lq - 1 : Xb - 1, Xbr = Xb + 1 == Lq ? 0 : Xb + 1;
                    const uint32_t ca = lds_code(lat, g, p, Y, X);
                    const uint32_t cb = lds_code(lat, g, 4 + pb, Yb, Xb);
                    const uint32_t bpack =
                        contrib_a(lds_code(lat, g, cAL, Y, p > 0 ? X : Xl)) +
                        contrib_a(lds_code(lat, g, cAR, Y, p < 3 ? X : Xr)) +
                        contrib_a(lds_code(lat, g, 4 + p, Y == 0 ? H - 1 : Y - 1, X)) +
                        contrib_a(lds_code(lat, g, 4 + p, Y, X)) +
                        contrib_b(lds_code(lat, g, cBL, Yb, pb > 0 ? Xb : Xbl)) +
                        contrib_b(lds_code(lat, g, cBR, Yb, pb < 3 ? Xb : Xbr)) +
                        contrib_b(lds_code(lat, g, pb, Yb, Xb)) +
                        contrib_b(lds_code(lat, g, pb, Yb + 1 == H ? 0 : Yb + 1, Xb));
                    const uint32_t s0 = ca | (cb << 2);
                    const uint32_t ns = pair_step(s0, bpack, h ? w.z : w.x, h ? w.w : w.y, s_trans, s_tab, packed);
                    if (ns != s0) {
                        atomicXor(&lat[g.word(p, Y, X)], ((ns ^ s0) & 3u) << (2 * (X & 15)));
                        atomicXor(&lat[g.word(4 + pb, Yb, Xb)], ((ns ^ s0) >> 2) << (2 * (Xb & 15)));
                    }
                }
                unpack_tracker(packed, tr);
            }
            __syncthreads();
        }
    }

    unstage_lattice(lat, d, g);
    if (threadIdx.x == 0) ((LatDesc *)(scr + kScrDesc))->next_sweep = d.next_sweep + my_sweeps;
    block_reduce_add<3>(tr, (unsigned long long *)(scr + kScrTrackBase));
}

template <int Q, bool Barrier>
__device__ __forceinline__ void word_sweeps(uint32_t *lat, uint32_t *sched, const LatDesc &d, uint32_t my_sweeps,
                                            const uint2 *s_tab, const uint4 *s_transd, int (&tr)[3])
{
    WordPhase f;
    f.W = d.L >> 6;
    f.H = d.L >> 1;
    f.Lq = d.L >> 2;
    f.magicW = f.W == 1 ? 0u : (uint32_t)((0x100000000ull + (uint64_t)f.W - 1u) / (uint64_t)f.W);
    f.key0 = d.key0;
    f.key1 = d.key1;
    const uint32_t csz = (uint32_t)f.H * (uint32_t)f.W;
    const uint32_t tasks = csz * (uint32_t)Q;
    // At most one task per thread (and Q >= 2, so that the held draws stay
    // few): each phase makes the next phase's draws of the thread's task
    // while its own table lookups are in flight.
    const bool pipe = Q >= 2 && tasks <= blockDim.x;
    u32x4 pre[kTaskCalls<Q>];
    if (pipe && threadIdx.x < tasks && my_sweeps > 0) {
        const uint32_t c0 = task_call0<Q>(f, threadIdx.x);
        const int q = (int)(threadIdx.x & (uint32_t)(Q - 1));
#pragma unroll
        for (int i = 0; i < kTaskCalls<Q>; ++i)
            pre[i] = philox4x32_10((uint32_t)d.next_sweep, 0u, c0 + (uint32_t)call_of_task<Q>(q, i),
                                   (uint32_t)(d.next_sweep >> 32), d.key0, d.key1);
    }
    for (uint32_t i = 0; i < my_sweeps; ++i) {
        const uint64_t s = d.next_sweep + i;
        const uint32_t *Wd = sched + 12u * (i & 1u);
        const int r = __builtin_amdgcn_readfirstlane(1 + (int)(((Wd[0] >> 8) * 3u) >> 24));
        f.s_lo = (uint32_t)s;
        f.s_hi = (uint32_t)(s >> 32);
        for (int p = 0; p < 4; ++p) {
            const int m = __builtin_amdgcn_readfirstlane((int)mulhi_u32(Wd[1 + 2 * p], (uint32_t)f.Lq));
            f.k = __builtin_amdgcn_readfirstlane((int)mulhi_u32(Wd[2 + 2 * p], (uint32_t)f.H));
            f.p = p;
            f.pb = (p + r) & 3;
            const int carry = (p + r) >> 2;
            f.dX = m + carry >= f.Lq ? m + carry - f.Lq : m + carry;
            f.oA0 = (uint32_t)p * csz;
            f.oAL = (uint32_t)(p > 0 ? p - 1 : 3) * csz;
            f.oAR = (uint32_t)(p < 3 ? p + 1 : 0) * csz;
            f.oAV = (uint32_t)(4 + p) * csz;
            f.oB0 = (uint32_t)(4 + f.pb) * csz;
            f.oBL = (uint32_t)(f.pb > 0 ? 4 + f.pb - 1 : 7) * csz;
            f.oBR = (uint32_t)(f.pb < 3 ? 4 + f.pb + 1 : 4) * csz;
            f.oBV = (uint32_t)f.pb * csz;
            // the next sweep's schedule words, into the other buffer (read
            // after this phase's barrier)
            if (p == 3 && threadIdx.x < 3 && i + 1 < my_sweeps) {
                const u32x4 w = philox4x32_10((uint32_t)(s + 1), kDomSchedule, threadIdx.x, (uint32_t)((s + 1) >> 32),
                                              d.key0, d.key1);
                uint32_t *o = sched + 12u * ((i + 1u) & 1u) + 4u * threadIdx.x;
                o[0] = w.x;
                o[1] = w.y;
                o[2] = w.z;
                o[3] = w.w;
            }
            if (pipe) {
                if (threadIdx.x < tasks)
                    word_task<Q, Barrier, kDrawPipe>(lat, f, threadIdx.x, s_tab, s_transd, tr, pre,
                                                     p < 3 ? s : s + 1, p < 3 ? p + 1 : 0);
            } else {
                for (uint32_t t = threadIdx.x; t < tasks; t += blockDim.x)
                    word_task<Q, Barrier>(lat, f, t, s_tab, s_transd, tr);
            }
            __syncthreads();
        }
    }
}

// This thread's share of the 7 observable sums of a 2-bit lattice in the
// class layout, read from st (global memory or the LDS copy).
__device__ __forceinline__ void obs_sums_2bit(const uint32_t *st, int L, long long (&v)[7])
{
    const uint32_t n = 8u * (uint32_t)(L >> 1) * (uint32_t)(L >> 6);
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) obs_word_2bit(st, L, i, v);
}

// This thread's share of a lattice's tracker slots (phase kernels) and, for
// thread 0, its tracker base (single-block kernels).
__device__ __forceinline__ void tracker_partial(const uint8_t *scr, long long (&t3)[3])
{
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
}

// MaxThreads = 512 serves blocks of up to 512 threads (measured faster: the
// compiler schedules for fewer waves per SIMD), 1024 the largest blocks.
template <int MaxThreads>
__global__ void __launch_bounds__(MaxThreads) k_sweep_lds_w(BatchArgs args)
{
    constexpr bool kBarrier = MaxThreads > 512;
    __shared__ uint2 s_tab[kDevTabEntries];
    __shared__ uint4 s_transd[kTransEntries];
    __shared__ uint32_t sched[24];
    extern __shared__ uint32_t lat[];
    uint8_t *scr = args.scratch[blockIdx.x];
    const LatDesc d = *(const LatDesc *)(scr + kScrDesc);
    const uint32_t my_sweeps = args.sweeps[blockIdx.x];
    if (threadIdx.x < 3) {
        const uint64_t s = d.next_sweep;
        const u32x4 w = philox4x32_10((uint32_t)s, kDomSchedule, threadIdx.x, (uint32_t)(s >> 32), d.key0, d.key1);
        sched[4 * threadIdx.x] = w.x;
        sched[4 * threadIdx.x + 1] = w.y;
        sched[4 * threadIdx.x + 2] = w.z;
        sched[4 * threadIdx.x + 3] = w.w;
    }
    LdsGeom g;
    g.L = d.L;
    g.Lq = d.L >> 2;
    g.H = d.L >> 1;
    g.Wp = d.L >> 6;
    g.csz = (uint32_t)g.H * g.Wp;
    stage_lattice(lat, d, g);
    {
        const uint2 *g_tab = (const uint2 *)(scr + kScrDevTab);
        const uint4 *g_transd = (const uint4 *)(scr + kScrTransD);
        for (int i = threadIdx.x; i < kDevTabEntries; i += blockDim.x) s_tab[i] = g_tab[i];
        for (int i = threadIdx.x; i < kTransEntries; i += blockDim.x) s_transd[i] = g_transd[i];
        __syncthreads();
    }

    // threads per a-word: the largest Q <= 8 with Q * (a-words) <= block size
    const uint32_t words = g.csz;
    int Q = 1;
    while (Q < 8 && words * (uint32_t)(2 * Q) <= blockDim.x) Q *= 2;
    int tr[3] = {0, 0, 0};
    switch (Q) {
    case 1: word_sweeps<1, kBarrier>(lat, sched, d, my_sweeps, s_tab, s_transd, tr); break;
    case 2: word_sweeps<2, kBarrier>(lat, sched, d, my_sweeps, s_tab, s_transd, tr); break;
    case 4: word_sweeps<4, kBarrier>(lat, sched, d, my_sweeps, s_tab, s_transd, tr); break;
    default: word_sweeps<8, kBarrier>(lat, sched, d, my_sweeps, s_tab, s_transd, tr); break;
    }
    if constexpr (MaxThreads <= 512) {
        if (args.obs_out) {
            // the interval's observables from the LDS copy, and the tracker
            // total as k_obs_batch would read it after this launch: the
            // slots, the base before this launch and this launch's own moves
            unsigned long long *o = args.obs_out + 10 * (size_t)blockIdx.x;
            long long t3[3] = {tr[0], tr[1], tr[2]};
            tracker_partial(scr, t3);
            long long v[7] = {0, 0, 0, 0, 0, 0, 0};
            obs_sums_2bit(lat, d.L, v);
            if (threadIdx.x < 10) o[threadIdx.x] = 0ull;
            __syncthreads();
            block_reduce_add<7>(v, o + 3);
            block_reduce_add<3>(t3, o);
        }
    }
    unstage_lattice(lat, d, g);
    if (threadIdx.x == 0) ((LatDesc *)(scr + kScrDesc))->next_sweep = d.next_sweep + my_sweeps;
    block_reduce_add<3>(tr, (unsigned long long *)(scr + kScrTrackBase));
}

__global__ void k_advance(LatDesc *desc, uint32_t sweeps)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) desc->next_sweep += sweeps;
}

// Observables of many lattices from their global state: block b reduces
// lattice b and writes (tracker, 7 sums) to out[10b ..].
__global__ void __launch_bounds__(256) k_obs_batch(BatchArgs args, unsigned long long *out)
{
    uint8_t *scr = args.scratch[blockIdx.x];
    const LatDesc d = *(const LatDesc *)(scr + kScrDesc);
    const int L = d.L;
    long long v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (d.enc == 0) {
        const int8_t *st = (const int8_t *)d.state;
        for (uint32_t i = threadIdx.x; i < (uint32_t)L * L; i += blockDim.x) {
            const int y = (int)(i / L), x = (int)(i - (uint32_t)y * L);
            const uint32_t c = (uint32_t)st[i];
            const uint32_t cr = (uint32_t)st[(size_t)y * L + (x + 1 == L ? 0 : x + 1)];
            const uint32_t cd = (uint32_t)st[(size_t)(y + 1 == L ? 0 : y + 1) * L + x];
            const int S = charge_of(c), G = spin_of(c), sg = ((x + y) & 1) ? -1 : 1;
            v[0] += S;
            v[1] += S * S;
            v[2] += S * (charge_of(cr) + charge_of(cd));
            v[3] += G * (spin_of(cr) + spin_of(cd));
            v[4] += G;
            v[5] += sg * G;
            v[6] += sg * S;
        }
    } else {
        obs_sums_2bit((const uint32_t *)d.state, L, v);
    }
    unsigned long long *o = out + 10 * (size_t)blockIdx.x;
    if (threadIdx.x < 10) o[threadIdx.x] = 0ull;
    __syncthreads();
    block_reduce_add<7>(v, o + 3);
    long long t3[3] = {0, 0, 0};
    tracker_partial(scr, t3);
    block_reduce_add<3>(t3, o);
}

}  // namespace

hipError_t init_kernel_attributes()
{
    // allow more than the default 64 KiB of dynamic LDS (L = 512 needs 64 KiB + tables)
    const int bytes = (int)(lds_state_words(kLdsMaxL) * 4u);
    hipError_t e = hipFuncSetAttribute((const void *)k_sweep_lds, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_sweep_lds_w<512>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_sweep_lds_w<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

hipError_t launch_sweep_lds(const BatchArgs &a, int max_L, int threads, bool word, hipStream_t s)
{
    // default block: per-site form, one thread per Philox call (two pairs);
    // word form, two threads per a-word (at least 256)
    const uint32_t sq = (uint32_t)max_L * (uint32_t)max_L;
    const uint32_t units = word ? std::max(256u, sq / 64u) : sq / 16u;
    uint32_t block = units < 1024u ? ((units + 63u) / 64u) * 64u : 1024u;
    if (threads > 0) block = (uint32_t)std::min(1024, std::max(64, threads / 64 * 64));
    if (block < 64u) block = 64u;
    const size_t lds = lds_state_words(max_L) * 4u;
    // a.obs_out: the 512-thread word form writes the observables itself;
    // the other forms are followed by the observables launch
    if (word && block <= 512u) {
        hipLaunchKernelGGL(k_sweep_lds_w<512>, dim3((unsigned)a.count), dim3(block), lds, s, a);
        return hipGetLastError();
    }
    if (word)
        hipLaunchKernelGGL(k_sweep_lds_w<1024>, dim3((unsigned)a.count), dim3(block), lds, s, a);
    else
        hipLaunchKernelGGL(k_sweep_lds, dim3((unsigned)a.count), dim3(block), lds, s, a);
    if (a.obs_out) hipLaunchKernelGGL(k_obs_batch, dim3((unsigned)a.count), dim3(256), 0, s, a, a.obs_out);
    return hipGetLastError();
}

hipError_t launch_advance(LatDesc *desc, uint32_t sweeps, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, desc, sweeps);
    return hipGetLastError();
}

hipError_t launch_observables_batch(const BatchArgs &a, unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_obs_batch, dim3((unsigned)a.count), dim3(256), 0, s, a, out);
    return hipGetLastError();
}

}  // namespace lat
