// Device helpers shared by the gfx950 kernels of the coupled-pair Metropolis
// sweep (arXiv:2301.11735, section 3.1 update, section 3.2 parallel form):
// table staging, the per-pair step, neighbour sums 16 sites at a time, the
// on-device schedule and block reductions.  Included by the .hip sources only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "philox.h"

namespace lat {
namespace {

constexpr uint32_t kM5 = 0x55555555u;  // bit 0 of every 2-bit field
constexpr uint32_t kM3 = 0x33333333u;  // low 2 bits of every nibble
constexpr uint32_t kM0F = 0x0F0F0F0Fu; // low nibble of every byte

constexpr int charge_c(int c) { return (c & 2) ? 1 - 2 * (c & 1) : 0; }

// Half the number of configurations k_q of the same-charge set, for every
// pair state st = code_a | code_b << 2 (2 bits per state): 3 for q = 0
// (k_q = 6), 2 for q = +-1 (k_q = 4), and 0 for the frozen |q| = 2 states,
// whose configuration index is then always 0 (their single entry is the null
// move).  j = floor(k_q u / 2^24) = floor((k_q/2) u / 2^23) for the 24-bit u.
constexpr uint32_t make_kq2()
{
    uint32_t v = 0;
    for (int st = 0; st < 16; ++st) {
        const int q = charge_c(st & 3) + charge_c(st >> 2);
        const uint32_t k2 = (q == 2 || q == -2) ? 0u : (q == 0 ? 3u : 2u);
        v |= k2 << (2 * st);
    }
    return v;
}
constexpr uint32_t kKq2 = make_kq2();

// k_q/2 of the 16 pairs of an aligned (a-word, b-word) couple, 2 bits per
// pair at the pairs' own bit positions: a pair is frozen when both sites are
// charges of one sign, has k_q = 4 when exactly one site is charged, and
// k_q = 6 otherwise.
__device__ __forceinline__ uint32_t word_kq2(uint32_t A, uint32_t B)
{
    const uint32_t ha = (A >> 1) & kM5, la = A & kM5, hb = (B >> 1) & kM5, lb = B & kM5;
    const uint32_t frozen = ha & hb & ~(la ^ lb);
    const uint32_t one = ha ^ hb;
    return (~(one | frozen) & kM5) | ((~frozen & kM5) << 1);
}

// Pair states of 8 pairs: nibble u of the result is code_a | code_b << 2 of
// pair 8*half + u, for the aligned (a-word, b-word) couple (A, B).  One byte
// permute gathers (A byte, B byte) pairs, then two swap stages interleave
// their nibbles and 2-bit fields.
__device__ __forceinline__ uint32_t pair_states8(uint32_t A, uint32_t B, int half)
{
    uint32_t x = __builtin_amdgcn_perm(B, A, half ? 0x07030602u : 0x05010400u);
    uint32_t t = (x ^ (x >> 4)) & 0x00F000F0u;
    x ^= t ^ (t << 4);
    t = (x ^ (x >> 2)) & 0x0C0C0C0Cu;
    return x ^ t ^ (t << 2);
}

__device__ __forceinline__ void stage_tables(uint2 *s_tab, uint2 *s_trans, const uint2 *__restrict__ g_tab,
                                             const uint2 *__restrict__ g_trans)
{
    for (int i = threadIdx.x; i < kDevTabEntries; i += blockDim.x) s_tab[i] = g_tab[i];
    for (int i = threadIdx.x; i < kTransEntries; i += blockDim.x) s_trans[i] = g_trans[i];
    __syncthreads();
}

// One coupled-pair Metropolis step (section 3.1).  bpack holds the neighbour
// sums (sumS_a+4, sumS_b+4, sumsig_a+4, sumsig_b+4) as bytes; uc picks the
// configuration j = floor(k_q * (uc >> 8) / 2^24); ua is the acceptance draw,
// compared as min(ua, 2^32-2) < thr so that the reserved "always" threshold
// 2^32-1 accepts every draw.  Returns the new pair state and adds the
// accepted move's packed triple to `packed`.
__device__ __forceinline__ uint32_t pair_step_k2(uint32_t st, uint32_t kq2, uint32_t bpack, uint32_t uc, uint32_t ua,
                                                 const uint2 *__restrict__ s_trans, const uint2 *__restrict__ s_tab,
                                                 uint32_t &packed)
{
    const uint32_t j = ((uc >> 8) * kq2) >> 23;
    const uint2 tr = s_trans[st * 6u + j];
    const int idx = __builtin_amdgcn_sdot4((int)tr.x, (int)bpack, (int)(tr.y & 0xFFFFu), false);
    const uint2 e = s_tab[idx];
    const bool acc = min(ua, 0xFFFFFFFEu) < e.x;
    packed += acc ? e.y : 0u;
    return acc ? (tr.y >> 16) : st;
}

// The same step with the delta form of the transition table: an accepted
// move ORs its code changes into dacc at the fields that `fields` selects
// (the pair's 2-bit field in the low half for site a and in the high half for
// site b); the caller XORs the accumulated changes into the codes.
__device__ __forceinline__ void pair_step_delta(uint32_t st, uint32_t kq2, uint32_t bpack, uint32_t uc, uint32_t ua,
                                                const uint4 *__restrict__ s_transd, const uint2 *__restrict__ s_tab,
                                                uint32_t fields, uint32_t &packed, uint32_t &dacc)
{
    const uint32_t j = ((uc >> 8) * kq2) >> 23;
    const uint4 tr = s_transd[st * 6u + j];
    const int idx = __builtin_amdgcn_sdot4((int)tr.x, (int)bpack, (int)tr.y, false);
    const uint2 e = s_tab[idx];
    const bool acc = min(ua, 0xFFFFFFFEu) < e.x;
    packed += acc ? e.y : 0u;
    dacc |= tr.z & (acc ? fields : 0u);
}

__device__ __forceinline__ uint32_t pair_step(uint32_t st, uint32_t bpack, uint32_t uc, uint32_t ua,
                                              const uint2 *__restrict__ s_trans, const uint2 *__restrict__ s_tab,
                                              uint32_t &packed)
{
    return pair_step_k2(st, (kKq2 >> (2u * st)) & 3u, bpack, uc, ua, s_trans, s_tab, packed);
}

// Per-thread tracker: counts and biased sums of the accepted triples.
__device__ __forceinline__ void unpack_tracker(uint32_t packed, int (&tr)[3])
{
    const int cnt = (int)(packed >> 27);
    tr[0] += (int)((packed >> 20) & 127u) - 2 * cnt;
    tr[1] += (int)((packed >> 10) & 1023u) - 16 * cnt;
    tr[2] += (int)(packed & 1023u) - 16 * cnt;
}

// Wave-wide sum by DPP (row reductions, then row broadcasts 15 and 31): the
// total ends in lane 63 and is returned to every lane.  Every lane of the
// wave must be active.
template <int Ctrl, int RowMask>
__device__ __forceinline__ int dpp_i32(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, Ctrl, RowMask, 0xF, false);
}
template <int Ctrl, int RowMask>
__device__ __forceinline__ long long dpp_i64(long long v)
{
    const int lo = dpp_i32<Ctrl, RowMask>((int)(uint32_t)v), hi = dpp_i32<Ctrl, RowMask>((int)((uint64_t)v >> 32));
    return (long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int dpp_step_sum(int v)
{
    v += dpp_i32<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp_i32<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += dpp_i32<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_i32<0x140, 0xF>(v);  // row_mirror
    v += dpp_i32<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_i32<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ long long dpp_step_sum(long long v)
{
    v += dpp_i64<0xB1, 0xF>(v);
    v += dpp_i64<0x4E, 0xF>(v);
    v += dpp_i64<0x141, 0xF>(v);
    v += dpp_i64<0x140, 0xF>(v);
    v += dpp_i64<0x142, 0xA>(v);
    v += dpp_i64<0x143, 0xC>(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)((uint64_t)v >> 32), 63);
    return (long long)(((uint64_t)hi << 32) | lo);
}

// Per-wave sums of K values, written to part[wave][*] by lane 0.  Full
// waves (blockDim a multiple of 64, the launch shapes of the sweep kernels)
// reduce by DPP; a partial wave falls back to shuffles.
template <int K, typename T>
__device__ __forceinline__ void wave_partials(T (&v)[K], T (*part)[K])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if ((blockDim.x & 63u) == 0) {
#pragma unroll
        for (int i = 0; i < K; ++i) v[i] = dpp_step_sum(v[i]);
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i)
            for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
    }
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < K; ++i) part[wave][i] = v[i];
}

// Block-level sum of K values added to dst[0..K): thread i < K sums value i
// over the block's waves and adds it with one atomic.
template <int K, typename T>
__device__ __forceinline__ void block_reduce_add(T (&v)[K], unsigned long long *dst)
{
    __shared__ T part[16][K];
    wave_partials<K, T>(v, part);
    __syncthreads();
    if (threadIdx.x < K) {
        const int nw = (blockDim.x + 63) >> 6;
        long long s = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w)
            if (w < nw) s += (long long)part[w][threadIdx.x];
        if (s != 0) atomicAdd(&dst[threadIdx.x], (unsigned long long)s);
    }
}

// Neighbour contribution of a code c to the packed sums: byte 0 (a side) or
// byte 1 (b side) gets 1+S(c), byte 2 or byte 3 gets 1+sigma(c); the values
// per code are the bytes of kVS = {1,1,2,0} and kVG = {2,0,1,1}.
constexpr uint32_t kVS = 0x00020101u;
constexpr uint32_t kVG = 0x01010002u;
__device__ __forceinline__ uint32_t contrib_a(uint32_t c) { return __builtin_amdgcn_perm(kVG, kVS, 0x0C040C00u + c * 0x00010001u); }
__device__ __forceinline__ uint32_t contrib_b(uint32_t c) { return __builtin_amdgcn_perm(kVG, kVS, 0x040C000Cu + c * 0x01000100u); }

// Schedule of sweep s (same definition as the host's): r in {1,2,3};
// phase p has D_p = (r + 4 m_p, 1 + 2 k_p).
__device__ __forceinline__ void device_schedule(int L, uint32_t k0, uint32_t k1, uint64_t s, int &r, int (&m)[4],
                                                int (&k)[4])
{
    uint32_t Wd[12];
#pragma unroll
    for (uint32_t t = 0; t < 3; ++t) {
        const u32x4 w = philox4x32_10((uint32_t)s, kDomSchedule, t, (uint32_t)(s >> 32), k0, k1);
        Wd[4 * t] = w.x;
        Wd[4 * t + 1] = w.y;
        Wd[4 * t + 2] = w.z;
        Wd[4 * t + 3] = w.w;
    }
    r = 1 + (int)(((Wd[0] >> 8) * 3u) >> 24);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        m[p] = (int)mulhi_u32(Wd[1 + 2 * p], (uint32_t)(L / 4));
        k[p] = (int)mulhi_u32(Wd[2 + 2 * p], (uint32_t)(L / 2));
    }
}

// Device-wide barrier between phases of the persistent kernels: every block
// arrives once per phase on a monotonic counter.  Release: every wave fences
// (a wave's fence waits only for its own stores and atomics), so the block's
// results are past the compute unit's caches before its arrival; acquire:
// the fence after the wait invalidates the caches the block reads through.
// The wait is bounded in time (kBarrierTimeoutTicks of the device's
// constant-rate wall clock, 0.2 s at its 100 MHz): then the block raises the
// error flag and goes on (results are then invalid and reported as an
// error), so no wave can spin for long.
__device__ __forceinline__ void grid_barrier(unsigned *counter, unsigned target, unsigned *err)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(counter, 1u);
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (wall_clock64() - t0 > kBarrierTimeoutTicks) {
                atomicOr(err, 1u);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// Word i of an array below 4 GiB (every lattice state is): a 32-bit byte
// offset from the base, so that a uniform base stays in scalar registers and
// no 64-bit address is formed per access.
__device__ __forceinline__ uint32_t word_at(const uint32_t *base, uint32_t i)
{
    return *(const uint32_t *)((const uint8_t *)base + (i << 2));
}
__device__ __forceinline__ void word_put(uint32_t *base, uint32_t i, uint32_t v)
{
    *(uint32_t *)((uint8_t *)base + (i << 2)) = v;
}

// The two words of the class row at word offset `row` that hold the 16 sites
// starting at class position xs (periodic); alignbit(hi, lo, 2 (xs mod 16))
// then gives the 16 sites (a shift of 0 gives lo).
__device__ __forceinline__ void load_pair(const uint32_t *__restrict__ st, uint32_t row, int W, int xs, uint32_t &lo,
                                          uint32_t &hi)
{
    const int jw = xs >> 4;
    lo = word_at(st, row + (uint32_t)jw);
    hi = word_at(st, row + (uint32_t)(jw + 1 == W ? 0 : jw + 1));
}

// 16 sites of the class row at word offset `row` of `st`, starting at class
// position xs (periodic).  32-bit offsets keep the base pointer uniform.
__device__ __forceinline__ uint32_t load16(const uint32_t *__restrict__ st, uint32_t row, int W, int xs)
{
    const int jw = xs >> 4, sh = xs & 15;
    const uint32_t w0 = word_at(st, row + (uint32_t)jw);
    const uint32_t w1 = word_at(st, row + (uint32_t)(jw + 1 == W ? 0 : jw + 1));
    return sh ? __builtin_amdgcn_alignbit(w1, w0, 2u * (uint32_t)sh) : w0;
}

// Neighbour sums of 16 sites from their 4 neighbour words, SWAR: per code
// the values 1+S in {0,1,2} and 1+sigma in {0,1,2} as 2-bit fields, split
// into even and odd sites so that the 4-term sums (at most 8) fit nibbles.
struct SideSums {
    uint32_t ES, OS, EG, OG;  // nibble u: sum over neighbours of site 2u (E) or 2u+1 (O)
};

// Adds one neighbour word's 16 values to the sums.
__device__ __forceinline__ void side_add(SideSums &s, uint32_t w)
{
    const uint32_t h = (w >> 1) & kM5, l = w & kM5;
    const uint32_t vS = ((h & ~l) << 1) | (h ^ kM5);        // code 2 -> 2, 3 -> 0, spins -> 1
    const uint32_t vG = (((h | l) ^ kM5) << 1) | h;          // code 0 -> 2, 1 -> 0, charges -> 1
    s.ES += vS & kM3;
    s.OS += (vS >> 2) & kM3;
    s.EG += vG & kM3;
    s.OG += (vG >> 2) & kM3;
}

// The sums over all four neighbour words at once, from three indicator
// planes per word (one bit per site, at the low bit of its field): h (a
// charge), P (charge +1) and U (spin +1).  Per site 1+S = 2P + 1 - h and
// 1+sigma = 2U + h, so over the four neighbours
//   4 + sum S = 4 + 2 sum P - sum h,   4 + sum sigma = 2 sum U + sum h.
// Two words' planes add without carry in 2-bit fields (at most 2); the two
// pair sums are then split into even and odd sites and added in nibbles (at
// most 4), and the nibble combinations stay within 0..8.
__device__ __forceinline__ SideSums side_sums(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3)
{
    uint32_t h[4], P[4], U[4];
    const uint32_t w[4] = {w0, w1, w2, w3};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h[i] = (w[i] >> 1) & kM5;
        P[i] = h[i] & ~w[i];
        U[i] = ~(h[i] | w[i]) & kM5;
    }
    const uint32_t h01 = h[0] + h[1], h23 = h[2] + h[3];
    const uint32_t P01 = P[0] + P[1], P23 = P[2] + P[3];
    const uint32_t U01 = U[0] + U[1], U23 = U[2] + U[3];
    const uint32_t hE = (h01 & kM3) + (h23 & kM3), hO = ((h01 >> 2) & kM3) + ((h23 >> 2) & kM3);
    const uint32_t PE = (P01 & kM3) + (P23 & kM3), PO = ((P01 >> 2) & kM3) + ((P23 >> 2) & kM3);
    const uint32_t UE = (U01 & kM3) + (U23 & kM3), UO = ((U01 >> 2) & kM3) + ((U23 >> 2) & kM3);
    constexpr uint32_t kFour = 0x44444444u;  // 4 in every nibble
    return SideSums{kFour + 2u * PE - hE, kFour + 2u * PO - hO, 2u * UE + hE, 2u * UO + hO};
}

// 4x4 byte transpose: out[k] = (r0.byte k, r1.byte k, r2.byte k, r3.byte k).
__device__ __forceinline__ void transpose4(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3, uint32_t &c0,
                                           uint32_t &c1, uint32_t &c2, uint32_t &c3)
{
    const uint32_t p01lo = __builtin_amdgcn_perm(r1, r0, 0x05010400u);
    const uint32_t p01hi = __builtin_amdgcn_perm(r1, r0, 0x07030602u);
    const uint32_t p23lo = __builtin_amdgcn_perm(r3, r2, 0x05010400u);
    const uint32_t p23hi = __builtin_amdgcn_perm(r3, r2, 0x07030602u);
    c0 = __builtin_amdgcn_perm(p23lo, p01lo, 0x05040100u);
    c1 = __builtin_amdgcn_perm(p23lo, p01lo, 0x07060302u);
    c2 = __builtin_amdgcn_perm(p23hi, p01hi, 0x05040100u);
    c3 = __builtin_amdgcn_perm(p23hi, p01hi, 0x07060302u);
}

// (r0.byte k, r1.byte k, r2.byte k, r3.byte k) with sel = k | (4 + k) << 8 | 0x0C0C0000.
__device__ __forceinline__ uint32_t gather_byte(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3, uint32_t sel)
{
    const uint32_t lo = __builtin_amdgcn_perm(r1, r0, sel);
    const uint32_t hi = __builtin_amdgcn_perm(r3, r2, sel);
    return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

// Observable sums: sum S, sum S^2, bonds S S, bonds sigma sigma, sum sigma,
// staggered sigma, staggered S.  Bonds (x,y)-(x+1,y) and (x,y)-(x,y+1).
__device__ __forceinline__ int spin_of(uint32_t c) { return (c & 2u) ? 0 : 1 - 2 * (int)(c & 1u); }
__device__ __forceinline__ int charge_of(uint32_t c) { return (c & 2u) ? 1 - 2 * (int)(c & 1u) : 0; }

// Block-level sum of K values written (not added) to dst[0..K): no atomics.
template <int K, typename T>
__device__ __forceinline__ void block_reduce_store(T (&v)[K], long long *dst)
{
    __shared__ T part[16][K];
    wave_partials<K, T>(v, part);
    __syncthreads();
    if (threadIdx.x < K) {
        const int nw = (blockDim.x + 63) >> 6;
        long long s = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w)
            if (w < nw) s += (long long)part[w][threadIdx.x];
        dst[threadIdx.x] = s;
    }
}

// Bond sums of 16 sites (h, l bit planes) with 16 partner sites (hp, lp):
// S S = +1 for equal charges, -1 for opposite; sigma sigma likewise for spins.
__device__ __forceinline__ void bond_sums(uint32_t h, uint32_t l, uint32_t hp, uint32_t lp, int &bSS, int &bss)
{
    const uint32_t diff = l ^ lp;
    const uint32_t cc = h & hp, mm = (h | hp) ^ kM5;  // both charged / both spins
    bSS += __popc(cc & ~diff) - __popc(cc & diff);
    bss += __popc(mm & ~diff) - __popc(mm & diff);
}

}  // namespace
}  // namespace lat
