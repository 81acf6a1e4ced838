// One a-word of a phase of the coupled-pair sweep (arXiv:2301.11735, section
// 3.1 update, section 3.2 parallel form), 16 pairs computed by Q cooperating
// lanes, on a lattice in the 2-bit class layout held in LDS or in global
// memory.  Shared by the batched kernels (lattice in LDS) and the
// multi-block phase kernels (lattice in global memory).  Included by the
// .hip sources only.
#pragma once

#include "device_common.h"

namespace lat {
namespace {

// Word-parallel form, for lattices with L % 64 == 0 in the 2-bit class
// layout (W = L/64 words per class row): a phase is computed 16 sites at a
// time as in the single-lattice phase kernel.  The 16 pairs of an a-word are split among Q threads (Q = 1, 2, 4
// or 8, chosen per lattice so that the block is filled): thread q of a word
// takes the Philox calls c with c % Q == q, i.e. sites 2c and 2c+1.
//
// Within a phase no updated site neighbours another updated site, so every
// neighbour word read is constant during the phase; the a-word and the two
// b-words a thread updates are shared with other threads only in bit fields
// that those threads neither read nor write (a reader of such a word
// extracts only its own fields), and the updates are applied as xor atomics
// of the changed bits (a plain store when Q = 1 for the a-word).  The same
// holds in LDS and in global memory, where the atomics act at the L2.

struct WordPhase {
    uint32_t oA0, oAL, oAR, oAV, oB0, oBL, oBR, oBV;  // class offsets (words)
    int W, H, Lq, dX, k, p, pb;
    uint32_t magicW;                                 // ceil(2^32 / W)
    uint32_t s_lo, s_hi, key0, key1;
};

// Lattice word accessors.  Coh = false: ordinary loads and stores (the
// lattice in LDS, or in global memory within one launch, whose end makes the
// writes visible).  Coh = true: loads and stores at device coherence, which
// no compute unit's or die's cache keeps stale, for the persistent kernels
// whose blocks exchange lattice words across device-wide barriers without
// cache write-back or invalidation.  Read-modify-writes are device-scope
// atomics in both cases.
template <bool Coh>
__device__ __forceinline__ uint32_t ldw(const uint32_t *p, uint32_t i)
{
    if constexpr (Coh)
        return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return p[i];
}
template <bool Coh>
__device__ __forceinline__ void stw(uint32_t *p, uint32_t i, uint32_t v)
{
    if constexpr (Coh)
        __hip_atomic_store(p + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        p[i] = v;
}
// 16 sites of the class row at word offset `row`, starting at class position
// xs (periodic), as load16 but through ldw.  Device-coherent reads load the
// second word only when xs starts mid-word (every caller's xs mod 16 depends
// on the phase and the schedule only, so the branch is uniform): at
// L = 1024 that saved 2.5% of a sweep.  Plain loads (LDS, or global memory
// within a launch) keep both, which measured slightly faster there.
template <bool Coh>
__device__ __forceinline__ uint32_t ld16(const uint32_t *st, uint32_t row, int W, int xs)
{
    const int jw = xs >> 4, sh = xs & 15;
    const uint32_t w0 = ldw<Coh>(st, row + (uint32_t)jw);
    if (Coh && sh == 0) return w0;
    const uint32_t w1 = ldw<Coh>(st, row + (uint32_t)(jw + 1 == W ? 0 : jw + 1));
    return sh ? __builtin_amdgcn_alignbit(w1, w0, 2u * (uint32_t)sh) : w0;
}

// Device-wide barrier for kernels whose lattice words are all accessed at
// device coherence (ldw/stw<true> and device-scope atomics), in two halves.
// Arrive: every wave waits for its own memory operations to complete, the
// block meets, and one thread arrives on the monotonic counter.  Wait: that
// thread waits for the others, and the block meets again.  No cache
// write-back or invalidation is needed.  Between the halves a block may do
// work that touches no lattice word.  The wait is bounded as in grid_barrier
// (time-out flag, then go on), by `limit` ticks of the device wall clock.
__device__ __forceinline__ void grid_arrive_coherent(unsigned *counter)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void grid_wait_coherent(unsigned *counter, unsigned target, unsigned *err,
                                                   long long limit = kBarrierTimeoutTicks)
{
    if (threadIdx.x == 0) {
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (wall_clock64() - t0 > limit) {
                atomicOr(err, 1u);
                break;
            }
        }
    }
    __syncthreads();
}
__device__ __forceinline__ void grid_barrier_coherent(unsigned *counter, unsigned target, unsigned *err)
{
    grid_arrive_coherent(counter);
    grid_wait_coherent(counter, target, err);
}

// The fields of WordPhase for phase p of a sweep with schedule (r, m, k), on
// a lattice of side L with key (key0, key1); s is the sweep index.
__device__ __forceinline__ void word_phase_setup(WordPhase &f, int L, uint32_t key0, uint32_t key1, uint64_t s,
                                                 int p, int r, const int (&mm)[4], const int (&kk)[4])
{
    f.W = L >> 6;
    f.H = L >> 1;
    f.Lq = L >> 2;
    f.magicW = f.W == 1 ? 0u : (uint32_t)((0x100000000ull + (uint64_t)f.W - 1u) / (uint64_t)f.W);
    f.key0 = key0;
    f.key1 = key1;
    f.s_lo = (uint32_t)s;
    f.s_hi = (uint32_t)(s >> 32);
    const uint32_t csz = (uint32_t)f.H * (uint32_t)f.W;
    f.k = kk[p];
    f.p = p;
    f.pb = (p + r) & 3;
    const int carry = (p + r) >> 2;
    f.dX = mm[p] + carry >= f.Lq ? mm[p] + carry - f.Lq : mm[p] + carry;
    f.oA0 = (uint32_t)p * csz;
    f.oAL = (uint32_t)(p > 0 ? p - 1 : 3) * csz;
    f.oAR = (uint32_t)(p < 3 ? p + 1 : 0) * csz;
    f.oAV = (uint32_t)(4 + p) * csz;
    f.oB0 = (uint32_t)(4 + f.pb) * csz;
    f.oBL = (uint32_t)(f.pb > 0 ? 4 + f.pb - 1 : 7) * csz;
    f.oBR = (uint32_t)(f.pb < 3 ? 4 + f.pb + 1 : 4) * csz;
    f.oBV = (uint32_t)f.pb * csz;
}

// Sum of the charges S and of the spins sigma of the 16 sites of a class
// word (2-bit codes: 0 sigma = +1, 1 sigma = -1, 2 S = +1, 3 S = -1).
__device__ __forceinline__ int charge_sum16(uint32_t w)
{
    const uint32_t h = (w >> 1) & kM5, l = w & kM5;
    return __popc(h & ~l) - __popc(h & l);
}
__device__ __forceinline__ int spin_sum16(uint32_t w)
{
    const uint32_t h = (w >> 1) & kM5, l = w & kM5;
    return __popc((h | l) ^ kM5) - __popc(l & ~h);
}

// Observable sums of class word i (16 sites) of a lattice of side L in the
// 2-bit class layout: sum S, sum S^2, the S S and sigma sigma bonds to the
// right and lower neighbours, sum sigma, and the staggered sums.  The right
// neighbours are the same word of the next class (or class 0 of the row,
// one site on), the lower ones the same word of the paired row class.
template <bool Coh = false>
__device__ __forceinline__ void obs_word_2bit(const uint32_t *st, int L, uint32_t i, long long (&v)[7])
{
    const int W = L >> 6, H = L >> 1, Lq = L >> 2;
    const uint32_t csz = (uint32_t)H * W;
    const int c = (int)(i / csz);
    const uint32_t rem = i - (uint32_t)c * csz;
    const int Y = (int)(rem / W), j = (int)(rem - (uint32_t)Y * W);
    const int cx = c & 3, cy = c >> 2;
    const uint32_t w = ldw<Coh>(st, i);
    const uint32_t wr = cx < 3 ? ldw<Coh>(st, i + csz)
                               : ld16<Coh>(st, (uint32_t)(4 * cy) * csz + (uint32_t)Y * W, W,
                                           16 * j + 1 == Lq ? 0 : 16 * j + 1);
    const uint32_t wd = cy == 0 ? ldw<Coh>(st, i + 4 * csz)
                                : ldw<Coh>(st, (uint32_t)cx * csz + (uint32_t)(Y + 1 == H ? 0 : Y + 1) * W + j);
    const uint32_t h = (w >> 1) & kM5, l = w & kM5;
    const int sumS = charge_sum16(w);
    const int sumG = spin_sum16(w);
    int bSS = 0, bss = 0;
    bond_sums(h, l, (wr >> 1) & kM5, wr & kM5, bSS, bss);
    bond_sums(h, l, (wd >> 1) & kM5, wd & kM5, bSS, bss);
    const int sg = ((cx + cy) & 1) ? -1 : 1;
    v[0] += sumS;
    v[1] += __popc(h);
    v[2] += bSS;
    v[3] += bss;
    v[4] += sumG;
    v[5] += sg * sumG;
    v[6] += sg * sumS;
}

// Barrier = true keeps the compiler from interleaving the Philox calls of a
// task (fewer live registers, needed at 1024 threads per block); without it
// the calls overlap each other's LDS table lookups.
// Value of the lane XOR lanes away (XOR = 1, 2: quad permutes; 4: any lane).
template <int XOR>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v)
{
    if constexpr (XOR == 1)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    else if constexpr (XOR == 2)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    else
        return (uint32_t)__shfl_xor((int)v, XOR, 64);
}

// Philox calls a task makes: all 8 of its word (Q = 1) or 8/Q of them.  The
// i-th is call_of_task(q, i), in the order word_task uses them.
template <int Q>
constexpr int kTaskCalls = Q == 1 ? 8 : 8 / Q;
template <int Q>
__device__ __forceinline__ int call_of_task(int q, int i)
{
    if constexpr (Q == 1) return i < 4 ? 2 * i : 2 * (i - 4) + 1;
    else if constexpr (Q == 2) return 2 * i + q;
    else return 2 * ((q >> 1) + 2 * i) + (q & 1);
}

// First counter word of a task's word (its a-word's first Philox call): the
// same in every phase, since each phase's a-class has the same shape.
template <int Q>
__device__ __forceinline__ uint32_t task_call0(const WordPhase &f, uint32_t task)
{
    constexpr int LOGQ = Q == 1 ? 0 : Q == 2 ? 1 : Q == 4 ? 2 : 3;
    const uint32_t wi = task >> LOGQ;
    const int Y = f.W == 1 ? (int)wi : (int)__umulhi(wi, f.magicW), j = (int)wi - Y * f.W;
    return (uint32_t)Y * (uint32_t)(f.Lq >> 1) + 8u * (uint32_t)j;
}

// Pipe (where the task's Philox draws come from): kDrawInPlace, computed
// here as they are used; kDrawPipe, this phase's given in pre[] and those of
// the next phase (sweep ns, phase np) computed here, between the phase's
// dependent LDS lookups, and returned in pre[]; kDrawGiven, this phase's
// given in pre[] (the caller makes the next phase's elsewhere).
// Combine (lattice in global memory): the Q lanes of a word first OR their
// code changes together (their fields are disjoint), then the word's first
// lane stores the a-word, which no other word reads or writes in the phase,
// and applies the two b-word changes as atomics; one store and two atomics
// per word instead of 3Q atomics.  Every lane of a word must be active.
// Coh: the lattice words are read and written through ldw/stw<true>.
// Obs (with Combine): the word's first lane also adds the changes of the
// spin sum, the staggered spin sum and the staggered charge sum over the
// word's a-sites and b-sites to dv[0..2] (the other observable sums are the
// tracker's: the charged-site count and the two bond sums change by exactly
// the accepted energy-change triples, and the charge sum does not change).
constexpr int kDrawInPlace = 0, kDrawPipe = 1, kDrawGiven = 2;
template <int Q, bool Barrier, int Pipe = kDrawInPlace, bool Combine = false, bool Coh = false, bool Obs = false>
__device__ __forceinline__ void word_task(uint32_t *lat, const WordPhase &f, uint32_t task, const uint2 *s_tab,
                                          const uint4 *s_transd, int (&tr)[3], u32x4 *pre = nullptr,
                                          uint64_t ns = 0, int np = 0, int *dv = nullptr)
{
    static_assert(!Obs || Combine, "the observable moves are taken where a word's changes are combined");
    constexpr int LOGQ = Q == 1 ? 0 : Q == 2 ? 1 : Q == 4 ? 2 : 3;
    const uint32_t wi = task >> LOGQ;
    const int q = (int)(task & (uint32_t)(Q - 1));
    const int W = f.W, H = f.H, Lq = f.Lq;
    const int Y = W == 1 ? (int)wi : (int)__umulhi(wi, f.magicW), j = (int)wi - Y * W;
    int Xb = 16 * j + f.dX;
    if (Xb >= Lq) Xb -= Lq;
    const int Yb = Y + f.k >= H ? Y + f.k - H : Y + f.k;
    const int xAL = f.p > 0 ? 16 * j : (j == 0 ? Lq - 1 : 16 * j - 1);
    const int xAR = f.p < 3 ? 16 * j : 16 * j + 1;
    const int xBL = f.pb > 0 ? Xb : (Xb == 0 ? Lq - 1 : Xb - 1);
    const int xBR = f.pb < 3 ? Xb : (Xb + 1 == Lq ? 0 : Xb + 1);
    const uint32_t ro = (uint32_t)Y * W, rob = (uint32_t)Yb * W;
    const uint32_t roU = (uint32_t)(Y == 0 ? H - 1 : Y - 1) * W;
    const uint32_t robD = (uint32_t)(Yb + 1 == H ? 0 : Yb + 1) * W;

    const uint32_t A0 = ldw<Coh>(lat, f.oA0 + ro + j);
    const uint32_t B0 = ld16<Coh>(lat, f.oB0 + rob, W, Xb);
    SideSums sa, sb;
    if constexpr (Q == 1) {
        sa = side_sums(ld16<Coh>(lat, f.oAL + ro, W, xAL), ld16<Coh>(lat, f.oAR + ro, W, xAR),
                       ldw<Coh>(lat, f.oAV + roU + j), ldw<Coh>(lat, f.oAV + ro + j));
        sb = side_sums(ld16<Coh>(lat, f.oBL + rob, W, xBL), ld16<Coh>(lat, f.oBR + rob, W, xBR),
                       ld16<Coh>(lat, f.oBV + rob, W, Xb), ld16<Coh>(lat, f.oBV + robD, W, Xb));
    } else {
        // The Q threads of a word are Q consecutive lanes.  Lanes of the
        // first half sum a-side neighbour words, the others b-side ones,
        // 8/Q words each; the partial sums (additive, nibble-wide) are
        // combined within the group and the two sides exchanged.
        const int side = q >= Q / 2;
        const int k0 = (q % (Q / 2)) * (8 / Q);
        const uint32_t base[4] = {side ? f.oBL + rob : f.oAL + ro, side ? f.oBR + rob : f.oAR + ro,
                                  side ? f.oBV + rob : f.oAV + roU, side ? f.oBV + robD : f.oAV + ro};
        const int xs[4] = {side ? xBL : xAL, side ? xBR : xAR, side ? Xb : 16 * j, side ? Xb : 16 * j};
        SideSums part{0u, 0u, 0u, 0u};
#pragma unroll
        for (int i = 0; i < 8 / Q; ++i) {
            const int kk = k0 + i;
            const uint32_t b = kk == 0 ? base[0] : kk == 1 ? base[1] : kk == 2 ? base[2] : base[3];
            const int x = kk == 0 ? xs[0] : kk == 1 ? xs[1] : kk == 2 ? xs[2] : xs[3];
            side_add(part, ld16<Coh>(lat, b, W, x));
        }
        SideSums full = part, other;
        if constexpr (Q >= 4) {
            full.ES += lane_xor<1>(part.ES);
            full.OS += lane_xor<1>(part.OS);
            full.EG += lane_xor<1>(part.EG);
            full.OG += lane_xor<1>(part.OG);
        }
        if constexpr (Q == 8) {
            full.ES += lane_xor<2>(full.ES);
            full.OS += lane_xor<2>(full.OS);
            full.EG += lane_xor<2>(full.EG);
            full.OG += lane_xor<2>(full.OG);
        }
        other.ES = lane_xor<Q / 2>(full.ES);
        other.OS = lane_xor<Q / 2>(full.OS);
        other.EG = lane_xor<Q / 2>(full.EG);
        other.OG = lane_xor<Q / 2>(full.OG);
        sa = side ? other : full;
        sb = side ? full : other;
    }

    const uint32_t call0 = (uint32_t)Y * (uint32_t)(Lq >> 1) + 8u * (uint32_t)j;
    // code changes of pairs 0-7 (dlo) and 8-15 (dhi): site a's in the low
    // half, site b's in the high half
    uint32_t dlo = 0u, dhi = 0u, packed = 0u;
    const uint32_t kq2w = word_kq2(A0, B0);
    u32x4 nxt[kTaskCalls<Q>];
    if constexpr (Pipe == kDrawPipe) {
#pragma unroll
        for (int i = 0; i < kTaskCalls<Q>; ++i)
            nxt[i] = philox4x32_10((uint32_t)ns, (uint32_t)np, call0 + (uint32_t)call_of_task<Q>(q, i),
                                   (uint32_t)(ns >> 32), f.key0, f.key1);
    }
    auto do_call = [&](int i, int c, uint32_t be, uint32_t bo, uint32_t &dacc) {
        const u32x4 w =
            Pipe != kDrawInPlace ? pre[i]
                                 : philox4x32_10(f.s_lo, (uint32_t)f.p, call0 + (uint32_t)c, f.s_hi, f.key0, f.key1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = 2 * c + h;
            const uint32_t s0 = ((A0 >> (2 * t)) & 3u) | (((B0 >> (2 * t)) & 3u) << 2);
            pair_step_delta(s0, (kq2w >> (2 * t)) & 3u, h ? bo : be, h ? w.z : w.x, h ? w.w : w.y, s_transd, s_tab,
                            0x00030003u << (2 * (t & 7)), packed, dacc);
        }
    };
    if constexpr (Q <= 2) {
#pragma unroll
        for (int hh = 0; hh < (Q == 1 ? 2 : 1); ++hh) {
            const int half = Q == 1 ? hh : q;
            const int sh = 4 * half;
            uint32_t ge[4], go[4];
            transpose4((sa.ES >> sh) & kM0F, (sb.ES >> sh) & kM0F, (sa.EG >> sh) & kM0F, (sb.EG >> sh) & kM0F,
                       ge[0], ge[1], ge[2], ge[3]);
            transpose4((sa.OS >> sh) & kM0F, (sb.OS >> sh) & kM0F, (sa.OG >> sh) & kM0F, (sb.OG >> sh) & kM0F,
                       go[0], go[1], go[2], go[3]);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {  // pairs 4kk .. 4kk+3
                const int slot = Q == 1 ? 4 * hh + kk : kk;
                if (kk < 2)
                    do_call(slot, 2 * kk + half, ge[kk], go[kk], dlo);
                else
                    do_call(slot, 2 * kk + half, ge[kk], go[kk], dhi);
                if (Barrier) __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
        const int half = q & 1, sh = 4 * half;
        const uint32_t rES0 = (sa.ES >> sh) & kM0F, rES1 = (sb.ES >> sh) & kM0F;
        const uint32_t rEG0 = (sa.EG >> sh) & kM0F, rEG1 = (sb.EG >> sh) & kM0F;
        const uint32_t rOS0 = (sa.OS >> sh) & kM0F, rOS1 = (sb.OS >> sh) & kM0F;
        const uint32_t rOG0 = (sa.OG >> sh) & kM0F, rOG1 = (sb.OG >> sh) & kM0F;
        uint32_t dx = 0u;  // Q = 8: pairs 4kk .. 4kk+3 of the one call, kk = q >> 1
#pragma unroll
        for (int i = 0; i < 8 / Q; ++i) {  // Q = 4: i = 0 covers pairs 0-7, i = 1 pairs 8-15
            const uint32_t kk = (uint32_t)(q >> 1) + 2u * (uint32_t)i;
            const uint32_t sel = kk | ((4u + kk) << 8) | 0x0C0C0000u;
            do_call(i, 2 * (int)kk + half, gather_byte(rES0, rES1, rEG0, rEG1, sel),
                    gather_byte(rOS0, rOS1, rOG0, rOG1, sel), Q == 8 ? dx : (i == 0 ? dlo : dhi));
        }
        if (Q == 8) {
            dlo = (q >> 1) < 2 ? dx : 0u;
            dhi = (q >> 1) < 2 ? 0u : dx;
        }
    }
    const uint32_t dA = __builtin_amdgcn_perm(dhi, dlo, 0x05040100u);
    const uint32_t dB = __builtin_amdgcn_perm(dhi, dlo, 0x07060302u);
    if constexpr (Pipe == kDrawPipe) {
#pragma unroll
        for (int i = 0; i < kTaskCalls<Q>; ++i) pre[i] = nxt[i];
    }
    unpack_tracker(packed, tr);
    const int jb = Xb >> 4, shb = Xb & 15;
    if constexpr (Combine) {
        uint32_t cA = dA, cB = dB;
        if constexpr (Q >= 2) {
            cA |= lane_xor<1>(cA);
            cB |= lane_xor<1>(cB);
        }
        if constexpr (Q >= 4) {
            cA |= lane_xor<2>(cA);
            cB |= lane_xor<2>(cB);
        }
        if constexpr (Q >= 8) {
            cA |= lane_xor<4>(cA);
            cB |= lane_xor<4>(cB);
        }
        if (q == 0) {
            if constexpr (Obs) {
                // staggered sign of a class (cx, cy): (-1)^(cx + cy); the
                // a-class is (p, 0), the b-class (pb, 1)
                const int gA = spin_sum16(A0 ^ cA) - spin_sum16(A0), gB = spin_sum16(B0 ^ cB) - spin_sum16(B0);
                const int sA = charge_sum16(A0 ^ cA) - charge_sum16(A0);
                const int sB = charge_sum16(B0 ^ cB) - charge_sum16(B0);
                const bool nA = f.p & 1, nB = !(f.pb & 1);
                dv[0] += gA + gB;
                dv[1] += (nA ? -gA : gA) + (nB ? -gB : gB);
                dv[2] += (nA ? -sA : sA) + (nB ? -sB : sB);
            }
            stw<Coh>(lat, f.oA0 + ro + j, A0 ^ cA);
            atomicXor(&lat[f.oB0 + rob + (uint32_t)jb], cB << (2 * shb));
            const uint32_t hi = shb ? cB >> (32 - 2 * shb) : 0u;
            atomicXor(&lat[f.oB0 + rob + (uint32_t)(jb + 1 == W ? 0 : jb + 1)], hi);
        }
    } else if constexpr (!Barrier) {
        // unconditional (an XOR with 0 changes nothing): branches on the
        // masks cost more than the LDS operations they would skip
        if (Q == 1)
            lat[f.oA0 + ro + j] = A0 ^ dA;
        else
            atomicXor(&lat[f.oA0 + ro + j], dA);
        atomicXor(&lat[f.oB0 + rob + (uint32_t)jb], dB << (2 * shb));
        const uint32_t hi = shb ? dB >> (32 - 2 * shb) : 0u;
        atomicXor(&lat[f.oB0 + rob + (uint32_t)(jb + 1 == W ? 0 : jb + 1)], hi);
    } else {
        // the 1024-thread build keeps the branches: without them it needs
        // more registers than 16 waves a compute unit leave
        if (Q == 1) {
            if (dA) lat[f.oA0 + ro + j] = A0 ^ dA;
        } else if (dA) {
            atomicXor(&lat[f.oA0 + ro + j], dA);
        }
        if (dB) {
            atomicXor(&lat[f.oB0 + rob + (uint32_t)jb], dB << (2 * shb));
            if (shb) {
                const uint32_t hi = dB >> (32 - 2 * shb);
                if (hi) atomicXor(&lat[f.oB0 + rob + (uint32_t)(jb + 1 == W ? 0 : jb + 1)], hi);
            }
        }
    }
}

}  // namespace
}  // namespace lat
