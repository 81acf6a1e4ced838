// gfx950 kernels of the coupled-pair Metropolis sweep (arXiv:2301.11735,
// section 3.1 update, section 3.2 parallel form) and of the observable
// reduction.  Integer-only: no floating point, no matrix cores.
//
// One phase updates the N/8 pairs a = (x, y), x = p (mod 4), y even, with
// partners b = a + D.  No updated site neighbours another updated site, so
// every pair reads only sites nobody writes in the phase and the pairs are
// independent; the phase equals their sequential composition.
//
// Per pair the work is table driven (both tables staged in LDS once per
// block): the pair state st = code_a | code_b<<2 and the choice j select a
// transition entry (section 3.1's same-charge sets); one v_dot4 of that
// entry with the packed neighbour sums gives the index of the move's
// energy-change triple in the threshold table; the acceptance test is one
// unsigned compare.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernels.h"
#include "philox.h"

namespace lat {
namespace {

constexpr uint32_t kM5 = 0x55555555u;  // bit 0 of every 2-bit field
constexpr uint32_t kM3 = 0x33333333u;  // low 2 bits of every nibble
constexpr uint32_t kM0F = 0x0F0F0F0Fu; // low nibble of every byte

constexpr int charge_c(int c) { return (c & 2) ? 1 - 2 * (c & 1) : 0; }

// Number of configurations k_q of the same-charge set for every pair state
// (3 bits per state): 6 for q = 0, 4 for q = +-1, and 1 for the frozen
// |q| = 2 states, whose single entry is the null move.
constexpr uint64_t make_kq()
{
    uint64_t v = 0;
    for (int st = 0; st < 16; ++st) {
        const int q = charge_c(st & 3) + charge_c(st >> 2);
        const uint64_t kq = (q == 2 || q == -2) ? 1 : (q == 0 ? 6 : 4);
        v |= kq << (3 * st);
    }
    return v;
}
constexpr uint64_t kKq = make_kq();

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
__device__ __forceinline__ uint32_t pair_step(uint32_t st, uint32_t bpack, uint32_t uc, uint32_t ua,
                                              const uint2 *__restrict__ s_trans, const uint2 *__restrict__ s_tab,
                                              uint32_t &packed)
{
    const uint32_t kq = (uint32_t)(kKq >> (3u * st)) & 7u;
    const uint32_t j = ((uc >> 8) * kq) >> 24;
    const uint2 tr = s_trans[st * 6u + j];
    const int idx = __builtin_amdgcn_sdot4((int)tr.x, (int)bpack, (int)(tr.y & 0xFFFFu), false);
    const uint2 e = s_tab[idx];
    const bool acc = min(ua, 0xFFFFFFFEu) < e.x;
    packed += acc ? e.y : 0u;
    return acc ? (tr.y >> 16) : st;
}

// Per-thread tracker: counts and biased sums of the accepted triples.
__device__ __forceinline__ void unpack_tracker(uint32_t packed, int (&tr)[3])
{
    const int cnt = (int)(packed >> 27);
    tr[0] += (int)((packed >> 20) & 127u) - 2 * cnt;
    tr[1] += (int)((packed >> 10) & 1023u) - 16 * cnt;
    tr[2] += (int)(packed & 1023u) - 16 * cnt;
}

template <int K, typename T>
__device__ __forceinline__ void block_reduce_add(T (&v)[K], unsigned long long *dst)
{
    __shared__ T part[16][K];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < K; ++i)
        for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < K; ++i) part[wave][i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            long long s = 0;
            for (int w = 0; w < nw; ++w) s += (long long)part[w][i];
            if (s != 0) atomicAdd(&dst[i], (unsigned long long)s);
        }
    }
}

// ---------------------------------------------------------------------------
// int8 layout: one code per byte, row-major.  Thread t owns Philox call t,
// i.e. pairs 2t and 2t+1 (words 0,1 and 2,3 of the call).
//
// Neighbour contribution of a code c to the packed sums: byte 0 (a side) or
// byte 1 (b side) gets 1+S(c), byte 2 or byte 3 gets 1+sigma(c); the values
// per code are the bytes of kVS = {1,1,2,0} and kVG = {2,0,1,1}.
constexpr uint32_t kVS = 0x00020101u;
constexpr uint32_t kVG = 0x01010002u;
__device__ __forceinline__ uint32_t contrib_a(uint32_t c) { return __builtin_amdgcn_perm(kVG, kVS, 0x0C040C00u + c * 0x00010001u); }
__device__ __forceinline__ uint32_t contrib_b(uint32_t c) { return __builtin_amdgcn_perm(kVG, kVS, 0x040C000Cu + c * 0x01000100u); }

__global__ void __launch_bounds__(256) k_phase_int8(PhaseArgs a)
{
    __shared__ uint2 s_tab[kDevTabEntries];
    __shared__ uint2 s_trans[kTransEntries];
    stage_tables(s_tab, s_trans, a.dev_tab, a.trans);
    const int L = a.L, Lq = L >> 2;
    const uint32_t n_calls = (uint32_t)L * (uint32_t)L / 16u;
    int8_t *st = (int8_t *)a.state;
    const int Dx = a.r + 4 * a.m, Dy = 1 + 2 * a.k;
    int tr[3] = {0, 0, 0};
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_calls; t += gridDim.x * blockDim.x) {
        const u32x4 w = philox4x32_10(a.s_lo, (uint32_t)a.p, t, a.s_hi, a.key0, a.key1);
        uint32_t packed = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t pi = 2u * t + (uint32_t)h;
            const int Y = (int)(pi / (uint32_t)Lq);
            const int x = 4 * ((int)pi - Y * Lq) + a.p, y = 2 * Y;
            int xb = x + Dx, yb = y + Dy;
            if (xb >= L) xb -= L;
            if (yb >= L) yb -= L;
            const int xl = x == 0 ? L - 1 : x - 1, xr = x == L - 1 ? 0 : x + 1;
            const int yu = y == 0 ? L - 1 : y - 1, yd = y == L - 1 ? 0 : y + 1;
            const int xbl = xb == 0 ? L - 1 : xb - 1, xbr = xb == L - 1 ? 0 : xb + 1;
            const int ybu = yb == 0 ? L - 1 : yb - 1, ybd = yb == L - 1 ? 0 : yb + 1;
            const size_t ia = (size_t)y * L + x, ib = (size_t)yb * L + xb;
            const uint32_t ca = (uint32_t)st[ia], cb = (uint32_t)st[ib];
            const uint32_t bpack =
                contrib_a(st[(size_t)y * L + xl]) + contrib_a(st[(size_t)y * L + xr]) +
                contrib_a(st[(size_t)yu * L + x]) + contrib_a(st[(size_t)yd * L + x]) +
                contrib_b(st[(size_t)yb * L + xbl]) + contrib_b(st[(size_t)yb * L + xbr]) +
                contrib_b(st[(size_t)ybu * L + xb]) + contrib_b(st[(size_t)ybd * L + xb]);
            const uint32_t s0 = ca | (cb << 2);
            const uint32_t ns = pair_step(s0, bpack, h ? w.z : w.x, h ? w.w : w.y, s_trans, s_tab, packed);
            if (ns != s0) {
                st[ia] = (int8_t)(ns & 3u);
                st[ib] = (int8_t)(ns >> 2);
            }
        }
        unpack_tracker(packed, tr);
    }
    block_reduce_add<3>(tr, a.track + 3 * (size_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// 2-bit layout (see lattice.h): class c = 4*(y&1) + (x&3) is an (L/2) x (L/4)
// array of sites, L/64 words per row, 16 sites per word.
//
// Thread (Y, j) owns word j of row Y of the a-class (p, 0): 16 pairs.  Their
// partners are the 16 consecutive b-class sites starting at class position
// 16j + dX of row Y + k, which straddle two b-words.  Each block holds whole
// class rows, so the b-row of a-row Y is read and written by one block only:
// after the block barrier, thread j assembles b-word jb+1 from its own new
// codes and those of thread j+1 (mod W), and every b-word has one writer.

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

// 16 sites of the class row at word offset `row` of `st`, starting at class
// position xs (periodic).  32-bit offsets keep the base pointer uniform.
__device__ __forceinline__ uint32_t load16(const uint32_t *__restrict__ st, uint32_t row, int W, int xs)
{
    const int jw = xs >> 4, sh = xs & 15;
    const uint32_t w0 = st[row + (uint32_t)jw];
    const uint32_t w1 = st[row + (uint32_t)(jw + 1 == W ? 0 : jw + 1)];
    return sh ? __builtin_amdgcn_alignbit(w1, w0, 2u * (uint32_t)sh) : w0;
}

// Neighbour sums of 16 sites from their 4 neighbour words, SWAR: per code
// the values 1+S in {0,1,2} and 1+sigma in {0,1,2} as 2-bit fields, split
// into even and odd sites so that the 4-term sums (at most 8) fit nibbles.
struct SideSums {
    uint32_t ES, OS, EG, OG;  // nibble u: sum over neighbours of site 2u (E) or 2u+1 (O)
};

__device__ __forceinline__ SideSums side_sums(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3)
{
    SideSums s{0u, 0u, 0u, 0u};
    const uint32_t ws[4] = {w0, w1, w2, w3};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t h = (ws[i] >> 1) & kM5, l = ws[i] & kM5;
        const uint32_t vS = ((h & ~l) << 1) | (h ^ kM5);        // code 2 -> 2, 3 -> 0, spins -> 1
        const uint32_t vG = (((h | l) ^ kM5) << 1) | h;          // code 0 -> 2, 1 -> 0, charges -> 1
        s.ES += vS & kM3;
        s.OS += (vS >> 2) & kM3;
        s.EG += vG & kM3;
        s.OG += (vG >> 2) & kM3;
    }
    return s;
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

// MinWaves > 1 asks the compiler to fit MinWaves waves per SIMD (at most
// 512/MinWaves VGPRs), e.g. two 1024-thread blocks per compute unit at 8.
// The ten words one thread reads for its 16 pairs: its a-word, the a-words'
// left/right/up/down neighbour words, and the same five for the 16 partners
// (the b-side words start mid-word and are funnel-shifted into place).
struct PairWords {
    uint32_t A0, AL, AR, AU, AD, B0, BL, BR, BU, BD;
};

// One phase of the 2-bit lattice by this block: row groups blockIdx.x,
// blockIdx.x + gridDim.x, ...  The tables are already staged in LDS.
__device__ __forceinline__ void phase_2bit(const PhaseArgs &a, int rows_per_block, const uint2 *__restrict__ s_tab,
                                           const uint2 *__restrict__ s_trans, uint32_t *xch, int (&tr)[3])
{

    const int L = a.L, W = L >> 6, H = L >> 1, Lq = L >> 2;
    const int rr = threadIdx.x / W, j = threadIdx.x - rr * W;
    const int n_groups = H / rows_per_block;
    uint32_t *st = (uint32_t *)a.state;
    const uint32_t csz = (uint32_t)H * (uint32_t)W;  // words per class; N/16 < 2^32
    const int p = a.p;
    const int pb = (p + a.r) & 3, carry = (p + a.r) >> 2;
    int dX = a.m + carry;
    if (dX >= Lq) dX -= Lq;
    int Xb = 16 * j + dX;
    if (Xb >= Lq) Xb -= Lq;
    const int jb = Xb >> 4, shb = Xb & 15;
    const uint32_t jw_out = (uint32_t)(jb + 1 == W ? 0 : jb + 1);
    const int j_next = j + 1 == W ? 0 : j + 1;
    // word offsets of the classes read on the a side and the b side
    const uint32_t oA0 = (uint32_t)p * csz;
    const uint32_t oAL = (uint32_t)(p > 0 ? p - 1 : 3) * csz;
    const uint32_t oAR = (uint32_t)(p < 3 ? p + 1 : 0) * csz;
    const uint32_t oAV = (uint32_t)(4 + p) * csz;
    const uint32_t oB0 = (uint32_t)(4 + pb) * csz;
    const uint32_t oBL = (uint32_t)(pb > 0 ? 4 + pb - 1 : 7) * csz;
    const uint32_t oBR = (uint32_t)(pb < 3 ? 4 + pb + 1 : 4) * csz;
    const uint32_t oBV = (uint32_t)pb * csz;
    const int xAL = p > 0 ? 16 * j : (j == 0 ? Lq - 1 : 16 * j - 1);
    const int xAR = p < 3 ? 16 * j : 16 * j + 1;
    const int xBL = pb > 0 ? Xb : (Xb == 0 ? Lq - 1 : Xb - 1);
    const int xBR = pb < 3 ? Xb : (Xb + 1 == Lq ? 0 : Xb + 1);

    auto row_of = [&](int g) { return g * rows_per_block + rr; };
    auto brow_of = [&](int Y) { return Y + a.k >= H ? Y + a.k - H : Y + a.k; };
    auto load_words = [&](int g) {
        const int Y = row_of(g), Yb = brow_of(Y);
        const uint32_t ro = (uint32_t)Y * W, rob = (uint32_t)Yb * W;
        const uint32_t roU = (uint32_t)(Y == 0 ? H - 1 : Y - 1) * W;
        const uint32_t robD = (uint32_t)(Yb + 1 == H ? 0 : Yb + 1) * W;
        PairWords w;
        w.A0 = st[oA0 + ro + j];
        w.AL = load16(st, oAL + ro, W, xAL);
        w.AR = load16(st, oAR + ro, W, xAR);
        w.AU = st[oAV + roU + j];
        w.AD = st[oAV + ro + j];
        w.B0 = load16(st, oB0 + rob, W, Xb);
        w.BL = load16(st, oBL + rob, W, xBL);
        w.BR = load16(st, oBR + rob, W, xBR);
        w.BU = load16(st, oBV + rob, W, Xb);
        w.BD = load16(st, oBV + robD, W, Xb);
        return w;
    };

    // Each group's words are fetched before the previous group is computed.
    // Every word read is either never written in this phase or written only
    // by this block in the iteration that owns it, after its read.
    int g = blockIdx.x;
    PairWords cur{};
    if (g < n_groups) cur = load_words(g);
    int buf = 0;
    for (; g < n_groups; g += gridDim.x, buf ^= 1) {
        const int gn = g + gridDim.x;
        PairWords nxt{};
        if (gn < n_groups) nxt = load_words(gn);
        const int Y = row_of(g), Yb = brow_of(Y);

        const SideSums sa = side_sums(cur.AL, cur.AR, cur.AU, cur.AD);
        const SideSums sb = side_sums(cur.BL, cur.BR, cur.BU, cur.BD);
        // bpack of site t = (sumS_a+4, sumS_b+4, sumsig_a+4, sumsig_b+4): site
        // t = 4k + g is byte k of nibble plane g (g = 0, 2: even sites, low and
        // high nibbles; g = 1, 3: odd sites).  Philox call c serves t = 2c and
        // 2c+1, so calls 0,2,4,6 need planes 0 and 1, calls 1,3,5,7 planes 2
        // and 3; handling them in that order keeps 8 packed words live.
        uint32_t Anew = 0u, Bnew = 0u, packed = 0u;
        const uint32_t call0 = (uint32_t)Y * (uint32_t)(Lq >> 1) + 8u * (uint32_t)j;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            uint32_t ge[4], go[4];
            const int sh = 4 * half;
            transpose4((sa.ES >> sh) & kM0F, (sb.ES >> sh) & kM0F, (sa.EG >> sh) & kM0F, (sb.EG >> sh) & kM0F,
                       ge[0], ge[1], ge[2], ge[3]);
            transpose4((sa.OS >> sh) & kM0F, (sb.OS >> sh) & kM0F, (sa.OG >> sh) & kM0F, (sb.OG >> sh) & kM0F,
                       go[0], go[1], go[2], go[3]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int c = 2 * k + half;
                const u32x4 w =
                    philox4x32_10(a.s_lo, (uint32_t)p, call0 + (uint32_t)c, a.s_hi, a.key0, a.key1);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int t = 2 * c + h;
                    const uint32_t s0 = ((cur.A0 >> (2 * t)) & 3u) | (((cur.B0 >> (2 * t)) & 3u) << 2);
                    const uint32_t ns = pair_step(s0, h ? go[k] : ge[k], h ? w.z : w.x, h ? w.w : w.y, s_trans,
                                                  s_tab, packed);
                    Anew |= (ns & 3u) << (2 * t);
                    Bnew |= (ns >> 2) << (2 * t);
                }
                // keep the scheduler from hoisting every Philox call at once
                // (register pressure decides how many waves fit per SIMD)
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        unpack_tracker(packed, tr);
        st[oA0 + (uint32_t)Y * W + j] = Anew;
        uint32_t *x = xch + buf * blockDim.x;
        x[threadIdx.x] = Bnew;
        __syncthreads();
        const uint32_t nb = x[rr * W + j_next];
        const uint32_t word = shb ? __builtin_amdgcn_alignbit(nb, Bnew, 32u - 2u * (uint32_t)shb) : nb;
        st[oB0 + (uint32_t)Yb * W + jw_out] = word;
        cur = nxt;
    }
    __syncthreads();  // the exchange buffer is reused by the next phase
}

template <int MinWaves>
__global__ void __launch_bounds__(1024, MinWaves) k_phase_2bit(PhaseArgs a, int rows_per_block)
{
    __shared__ uint2 s_tab[kDevTabEntries];
    __shared__ uint2 s_trans[kTransEntries];
    extern __shared__ uint32_t xch[];  // 2 x blockDim (double buffered)
    stage_tables(s_tab, s_trans, a.dev_tab, a.trans);
    int tr[3] = {0, 0, 0};
    phase_2bit(a, rows_per_block, s_tab, s_trans, xch, tr);
    block_reduce_add<3>(tr, a.track + 3 * (size_t)blockIdx.x);
}

// Device-wide barrier between phases of the persistent kernel: every block
// arrives once per phase on a monotonic counter.  Release: the fence writes
// this block's results back past the compute unit's caches before the
// arrival; acquire: the fence after the wait invalidates them.  The wait is
// bounded: after about 2^24 polls the block raises the error flag and goes
// on (results are then invalid and reported as an error), so no wave can
// spin forever.
__device__ __forceinline__ void grid_barrier(unsigned *counter, unsigned target, unsigned *err)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(counter, 1u);
        unsigned polls = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++polls > (1u << 24)) {
                atomicOr(err, 1u);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// Persistent form: `sweeps` sweeps from sweep a.s_lo|a.s_hi in one launch of
// co-resident blocks (cooperative launch), tables staged once, schedules
// computed on the device, a device-wide barrier after every phase.
template <int MinWaves>
__global__ void __launch_bounds__(1024, MinWaves) k_sweeps_2bit(PhaseArgs a, int rows_per_block, uint32_t sweeps,
                                                                unsigned *counter, unsigned *err)
{
    __shared__ uint2 s_tab[kDevTabEntries];
    __shared__ uint2 s_trans[kTransEntries];
    extern __shared__ uint32_t xch[];
    stage_tables(s_tab, s_trans, a.dev_tab, a.trans);
    int tr[3] = {0, 0, 0};
    const uint64_t s0 = ((uint64_t)a.s_hi << 32) | a.s_lo;
    unsigned arrivals = 0;
    for (uint32_t i = 0; i < sweeps; ++i) {
        const uint64_t s = s0 + i;
        int r, mm[4], kk[4];
        device_schedule(a.L, a.key0, a.key1, s, r, mm, kk);
        PhaseArgs b = a;
        b.s_lo = (uint32_t)s;
        b.s_hi = (uint32_t)(s >> 32);
        b.r = r;
        for (int p = 0; p < 4; ++p) {
            b.p = p;
            b.m = mm[p];
            b.k = kk[p];
            phase_2bit(b, rows_per_block, s_tab, s_trans, xch, tr);
            arrivals += gridDim.x;
            grid_barrier(counter, arrivals, err);
        }
    }
    block_reduce_add<3>(tr, a.track + 3 * (size_t)blockIdx.x);
}



// ---------------------------------------------------------------------------
__global__ void k_zero_i64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Observable sums: sum S, sum S^2, bonds S S, bonds sigma sigma, sum sigma,
// staggered sigma, staggered S.  Bonds (x,y)-(x+1,y) and (x,y)-(x,y+1).
__device__ __forceinline__ int spin_of(uint32_t c) { return (c & 2u) ? 0 : 1 - 2 * (int)(c & 1u); }
__device__ __forceinline__ int charge_of(uint32_t c) { return (c & 2u) ? 1 - 2 * (int)(c & 1u) : 0; }

// Block-level sum of K values written (not added) to dst[0..K): no atomics.
template <int K, typename T>
__device__ __forceinline__ void block_reduce_store(T (&v)[K], long long *dst)
{
    __shared__ long long part[16][K];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < K; ++i)
        for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < K; ++i) part[wave][i] = (long long)v[i];
    __syncthreads();
    if (threadIdx.x < K) {
        const int nw = (blockDim.x + 63) >> 6;
        long long s = 0;
        for (int w = 0; w < nw; ++w) s += part[w][threadIdx.x];
        dst[threadIdx.x] = s;
    }
}

__global__ void __launch_bounds__(1024) k_obs_int8(const int8_t *__restrict__ st, int L, long long *slots)
{
    long long v[7] = {0, 0, 0, 0, 0, 0, 0};
    const uint32_t N = (uint32_t)L * (uint32_t)L;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int y = (int)(i / (uint32_t)L), x = (int)(i - (uint32_t)y * L);
        const uint32_t c = (uint32_t)st[i];
        const uint32_t cr = (uint32_t)st[(uint32_t)y * L + (x + 1 == L ? 0 : x + 1)];
        const uint32_t cd = (uint32_t)st[(uint32_t)(y + 1 == L ? 0 : y + 1) * L + x];
        const int S = charge_of(c), G = spin_of(c), sg = ((x + y) & 1) ? -1 : 1;
        v[0] += S;
        v[1] += S * S;
        v[2] += S * (charge_of(cr) + charge_of(cd));
        v[3] += G * (spin_of(cr) + spin_of(cd));
        v[4] += G;
        v[5] += sg * G;
        v[6] += sg * S;
    }
    block_reduce_store<7>(v, slots + 7 * (size_t)blockIdx.x);
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

// One class word (16 sites) per thread: its right neighbours are the same
// word of the next class (or class 0 one site on), its lower neighbours the
// same word of the paired row class.  Popcounts over the bit planes.
__global__ void __launch_bounds__(1024) k_obs_2bit(const uint32_t *__restrict__ st, int L, long long *slots)
{
    long long v[7] = {0, 0, 0, 0, 0, 0, 0};
    const uint32_t W = (uint32_t)L >> 6, H = (uint32_t)L >> 1, Lq = (uint32_t)L >> 2;
    const uint32_t csz = H * W, nwords = 8u * csz;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x) {
        const uint32_t c = i / csz, rem = i - c * csz;
        const uint32_t Y = rem / W, j = rem - Y * W;
        const uint32_t cx = c & 3u, cy = c >> 2;
        const uint32_t w = st[i];
        const uint32_t wr = cx < 3 ? st[i + csz] : load16(st, 4u * cy * csz + Y * W, (int)W, 16 * j + 1 == Lq ? 0 : (int)(16 * j + 1));
        const uint32_t wd = cy == 0 ? st[i + 4 * csz] : st[cx * csz + (Y + 1 == H ? 0 : Y + 1) * W + j];
        const uint32_t h = (w >> 1) & kM5, l = w & kM5;
        const int sumS = __popc(h & ~l) - __popc(h & l);
        const int sumG = __popc((h | l) ^ kM5) - __popc(l & ~h);
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
    block_reduce_store<7>(v, slots + 7 * (size_t)blockIdx.x);
}

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
    const uint32_t nwords = 8u * g.csz;

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

// ---------------------------------------------------------------------------
// Batched sweeps, word-parallel form, for lattices with L % 64 == 0: the LDS
// copy has the global 2-bit class layout (W = L/64 words per class row), and
// a phase is computed 16 sites at a time as in the single-lattice phase
// kernel.  The 16 pairs of an a-word are split among Q threads (Q = 1, 2, 4
// or 8, chosen per lattice so that the block is filled): thread q of a word
// takes the Philox calls c with c % Q == q, i.e. sites 2c and 2c+1.
//
// Within a phase no updated site neighbours another updated site, so every
// neighbour word read is constant during the phase; the a-word and the two
// b-words a thread updates are shared with other threads only in bit fields
// that those threads neither read nor write, and the updates are applied as
// LDS xor atomics of the changed bits (a plain store when Q = 1 for the a-word).

// (r0.byte k, r1.byte k, r2.byte k, r3.byte k) with sel = k | (4 + k) << 8 | 0x0C0C0000.
__device__ __forceinline__ uint32_t gather_byte(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3, uint32_t sel)
{
    const uint32_t lo = __builtin_amdgcn_perm(r1, r0, sel);
    const uint32_t hi = __builtin_amdgcn_perm(r3, r2, sel);
    return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

struct WordPhase {
    uint32_t oA0, oAL, oAR, oAV, oB0, oBL, oBR, oBV;  // class offsets (words)
    int W, H, Lq, dX, k, p, pb;
    uint32_t magicW;                                 // ceil(2^32 / W)
    uint32_t s_lo, s_hi, key0, key1;
};

// Barrier = true keeps the compiler from interleaving the Philox calls of a
// task (fewer live registers, needed at 1024 threads per block); without it
// the calls overlap each other's LDS table lookups.
template <int Q, bool Barrier>
__device__ __forceinline__ void word_task(uint32_t *lat, const WordPhase &f, uint32_t task, const uint2 *s_tab,
                                          const uint2 *s_trans, int (&tr)[3])
{
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

    const uint32_t A0 = lat[f.oA0 + ro + j];
    const uint32_t B0 = load16(lat, f.oB0 + rob, W, Xb);
    const SideSums sa = side_sums(load16(lat, f.oAL + ro, W, xAL), load16(lat, f.oAR + ro, W, xAR),
                                  lat[f.oAV + roU + j], lat[f.oAV + ro + j]);
    const SideSums sb = side_sums(load16(lat, f.oBL + rob, W, xBL), load16(lat, f.oBR + rob, W, xBR),
                                  load16(lat, f.oBV + rob, W, Xb), load16(lat, f.oBV + robD, W, Xb));

    const uint32_t call0 = (uint32_t)Y * (uint32_t)(Lq >> 1) + 8u * (uint32_t)j;
    uint32_t dA = 0u, dB = 0u, packed = 0u;
    auto do_call = [&](int c, uint32_t be, uint32_t bo) {
        const u32x4 w = philox4x32_10(f.s_lo, (uint32_t)f.p, call0 + (uint32_t)c, f.s_hi, f.key0, f.key1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = 2 * c + h;
            const uint32_t s0 = ((A0 >> (2 * t)) & 3u) | (((B0 >> (2 * t)) & 3u) << 2);
            const uint32_t ns = pair_step(s0, h ? bo : be, h ? w.z : w.x, h ? w.w : w.y, s_trans, s_tab, packed);
            const uint32_t dd = ns ^ s0;
            dA |= (dd & 3u) << (2 * t);
            dB |= (dd >> 2) << (2 * t);
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
            for (int kk = 0; kk < 4; ++kk) {
                do_call(2 * kk + half, ge[kk], go[kk]);
                if (Barrier) __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
        const int half = q & 1, sh = 4 * half;
        const uint32_t rES0 = (sa.ES >> sh) & kM0F, rES1 = (sb.ES >> sh) & kM0F;
        const uint32_t rEG0 = (sa.EG >> sh) & kM0F, rEG1 = (sb.EG >> sh) & kM0F;
        const uint32_t rOS0 = (sa.OS >> sh) & kM0F, rOS1 = (sb.OS >> sh) & kM0F;
        const uint32_t rOG0 = (sa.OG >> sh) & kM0F, rOG1 = (sb.OG >> sh) & kM0F;
#pragma unroll
        for (int i = 0; i < 8 / Q; ++i) {
            const uint32_t kk = (uint32_t)(q >> 1) + 2u * (uint32_t)i;
            const uint32_t sel = kk | ((4u + kk) << 8) | 0x0C0C0000u;
            do_call(2 * (int)kk + half, gather_byte(rES0, rES1, rEG0, rEG1, sel),
                    gather_byte(rOS0, rOS1, rOG0, rOG1, sel));
        }
    }
    unpack_tracker(packed, tr);
    if (Q == 1) {
        if (dA) lat[f.oA0 + ro + j] = A0 ^ dA;
    } else if (dA) {
        atomicXor(&lat[f.oA0 + ro + j], dA);
    }
    if (dB) {
        const int jb = Xb >> 4, shb = Xb & 15;
        atomicXor(&lat[f.oB0 + rob + (uint32_t)jb], dB << (2 * shb));
        if (shb) {
            const uint32_t hi = dB >> (32 - 2 * shb);
            if (hi) atomicXor(&lat[f.oB0 + rob + (uint32_t)(jb + 1 == W ? 0 : jb + 1)], hi);
        }
    }
}

template <int Q, bool Barrier>
__device__ __forceinline__ void word_sweeps(uint32_t *lat, uint32_t *sched, const LatDesc &d, uint32_t my_sweeps,
                                            const uint2 *s_tab, const uint2 *s_trans, int (&tr)[3])
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
            for (uint32_t t = threadIdx.x; t < tasks; t += blockDim.x) word_task<Q, Barrier>(lat, f, t, s_tab, s_trans, tr);
            __syncthreads();
        }
    }
}

// MaxThreads = 512 serves blocks of up to 512 threads (measured faster: the
// compiler schedules for fewer waves per SIMD), 1024 the largest blocks.
template <int MaxThreads>
__global__ void __launch_bounds__(MaxThreads) k_sweep_lds_w(BatchArgs args)
{
    constexpr bool kBarrier = MaxThreads > 512;
    __shared__ uint2 s_tab[kDevTabEntries];
    __shared__ uint2 s_trans[kTransEntries];
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
    stage_tables(s_tab, s_trans, (const uint2 *)(scr + kScrDevTab), (const uint2 *)(scr + kScrTrans));

    // threads per a-word: the largest Q <= 8 with Q * (a-words) <= block size
    const uint32_t words = g.csz;
    int Q = 1;
    while (Q < 8 && words * (uint32_t)(2 * Q) <= blockDim.x) Q *= 2;
    int tr[3] = {0, 0, 0};
    switch (Q) {
    case 1: word_sweeps<1, kBarrier>(lat, sched, d, my_sweeps, s_tab, s_trans, tr); break;
    case 2: word_sweeps<2, kBarrier>(lat, sched, d, my_sweeps, s_tab, s_trans, tr); break;
    case 4: word_sweeps<4, kBarrier>(lat, sched, d, my_sweeps, s_tab, s_trans, tr); break;
    default: word_sweeps<8, kBarrier>(lat, sched, d, my_sweeps, s_tab, s_trans, tr); break;
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
        const uint32_t *st = (const uint32_t *)d.state;
        const int W = L >> 6, H = L >> 1, Lq = L >> 2;
        const uint32_t csz = (uint32_t)H * W;
        for (uint32_t i = threadIdx.x; i < 8u * csz; i += blockDim.x) {
            const int c = (int)(i / csz);
            const uint32_t rem = i - (uint32_t)c * csz;
            const int Y = (int)(rem / W), j = (int)(rem - (uint32_t)Y * W);
            const int cx = c & 3, cy = c >> 2;
            const uint32_t w = st[i];
            const uint32_t wr = cx < 3 ? st[i + csz]
                                       : load16(st, (uint32_t)(4 * cy) * csz + (uint32_t)Y * W, W,
                                                16 * j + 1 == Lq ? 0 : 16 * j + 1);
            const uint32_t wd = cy == 0 ? st[i + 4 * csz] : st[(uint32_t)cx * csz + (uint32_t)(Y + 1 == H ? 0 : Y + 1) * W + j];
            const uint32_t h = (w >> 1) & kM5, l = w & kM5;
            const int sumS = __popc(h & ~l) - __popc(h & l);
            const int sumG = __popc((h | l) ^ kM5) - __popc(l & ~h);
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
    }
    unsigned long long *o = out + 10 * (size_t)blockIdx.x;
    if (threadIdx.x < 10) o[threadIdx.x] = 0ull;
    __syncthreads();
    block_reduce_add<7>(v, o + 3);
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
    block_reduce_add<3>(t3, o);
}

// Totals of one lattice: tracker = base triple + every tracker slot;
// observables = the first n_obs observable slots.
__global__ void __launch_bounds__(256) k_fold_sums(uint8_t *scr, int n_obs)
{
    long long t[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const long long *slots = (const long long *)(scr + kScrSlots);
    for (int i = threadIdx.x; i < kMaxSlots; i += blockDim.x) {
        t[0] += slots[3 * i];
        t[1] += slots[3 * i + 1];
        t[2] += slots[3 * i + 2];
    }
    if (threadIdx.x == 0) {
        const long long *base = (const long long *)(scr + kScrTrackBase);
        t[0] += base[0];
        t[1] += base[1];
        t[2] += base[2];
    }
    const long long *os = (const long long *)(scr + kScrObsSlots);
    for (int i = threadIdx.x; i < n_obs; i += blockDim.x)
#pragma unroll
        for (int k = 0; k < 7; ++k) t[3 + k] += os[7 * i + k];
    block_reduce_store<10>(t, (long long *)(scr + kScrTrack));
}

int g_num_cus = 0;

int num_cus()
{
    if (g_num_cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            g_num_cus = n;
        else
            g_num_cus = 256;
    }
    return g_num_cus;
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_phase_int8(const PhaseArgs &a, hipStream_t s)
{
    const uint32_t n_calls = (uint32_t)a.L * (uint32_t)a.L / 16u;
    const uint32_t block = 256;
    uint32_t grid = (n_calls + block - 1) / block;
    uint32_t cap = 4u * (uint32_t)num_cus();
    if (cap > (uint32_t)kMaxSlots) cap = (uint32_t)kMaxSlots;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(k_phase_int8, dim3(grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

// Rows per block: a power of two <= 32 (so it divides the L/2 = 32W rows);
// by default the largest giving at most 1024 threads.  Every block holds
// whole class rows.  One such block per compute unit stages the LDS tables
// once per launch and was the fastest shape measured at L = 8192.
static int rows_per_block_2bit(int W, int requested)
{
    const int cap = requested > 0 ? requested : 32;
    int r = 1;
    while (r < 32 && 2 * r <= cap && 2 * r * W <= 1024) r *= 2;
    return r;
}

hipError_t launch_phase_2bit(const PhaseArgs &a, const Tuning2Bit &t, hipStream_t s)
{
    const int W = a.L >> 6, H = a.L >> 1;
    const int R = rows_per_block_2bit(W, t.rows_per_block);
    const int block = R * W;
    int grid = H / R;
    const int bpc = t.blocks_per_cu > 0 ? t.blocks_per_cu : 1;
    if (grid > bpc * num_cus()) grid = bpc * num_cus();
    if (grid > kMaxSlots) grid = kMaxSlots;
    if (t.waves_hint >= 8)
        hipLaunchKernelGGL(k_phase_2bit<8>, dim3(grid), dim3(block), (size_t)block * 8u, s, a, R);
    else
        hipLaunchKernelGGL(k_phase_2bit<1>, dim3(grid), dim3(block), (size_t)block * 8u, s, a, R);
    return hipGetLastError();
}

bool persistent_2bit_supported(int L, const Tuning2Bit &t, int *grid_out, int *rows_out)
{
    int dev = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    const int W = L >> 6, R = rows_per_block_2bit(W, t.rows_per_block), block = R * W;
    int per_cu = 0;
    const void *fn = t.waves_hint >= 8 ? (const void *)k_sweeps_2bit<8> : (const void *)k_sweeps_2bit<1>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, (size_t)block * 8u) != hipSuccess ||
        per_cu < 1)
        return false;
    const int want = t.blocks_per_cu > 0 ? t.blocks_per_cu : 1;
    *grid_out = std::min(std::min(per_cu, want) * num_cus(), kMaxSlots);
    *rows_out = R;
    return true;
}

hipError_t launch_sweeps_2bit(const PhaseArgs &a, const Tuning2Bit &t, uint32_t sweeps, unsigned *counter,
                              unsigned *err, hipStream_t s)
{
    int grid = 0, R = 0;
    if (!persistent_2bit_supported(a.L, t, &grid, &R)) return hipErrorNotSupported;
    const int block = R * (a.L >> 6);
    hipError_t e = launch_zero_i64((unsigned long long *)counter, 1, s);  // counter (and the word after it)
    if (e != hipSuccess) return e;
    PhaseArgs args = a;
    int rows = R;
    uint32_t n = sweeps;
    void *kargs[] = {&args, &rows, &n, &counter, &err};
    const void *fn = t.waves_hint >= 8 ? (const void *)k_sweeps_2bit<8> : (const void *)k_sweeps_2bit<1>;
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), kargs, (size_t)block * 8u, s);
}


hipError_t launch_zero_i64(unsigned long long *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_i64, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_observables(uint8_t *scratch, const void *state, int L, int encoding, hipStream_t s)
{
    const uint32_t units = encoding == 0 ? (uint32_t)L * L : (uint32_t)L * L / 16u;
    uint32_t grid = (units + 1023u) / 1024u;
    if (grid > (uint32_t)kMaxObsSlots) grid = (uint32_t)kMaxObsSlots;
    long long *slots = (long long *)(scratch + kScrObsSlots);
    if (encoding == 0)
        hipLaunchKernelGGL(k_obs_int8, dim3(grid), dim3(1024), 0, s, (const int8_t *)state, L, slots);
    else
        hipLaunchKernelGGL(k_obs_2bit, dim3(grid), dim3(1024), 0, s, (const uint32_t *)state, L, slots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold_sums, dim3(1), dim3(256), 0, s, scratch, (int)grid);
    return hipGetLastError();
}

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
    if (word && block <= 512u)
        hipLaunchKernelGGL(k_sweep_lds_w<512>, dim3((unsigned)a.count), dim3(block), lds, s, a);
    else if (word)
        hipLaunchKernelGGL(k_sweep_lds_w<1024>, dim3((unsigned)a.count), dim3(block), lds, s, a);
    else
        hipLaunchKernelGGL(k_sweep_lds, dim3((unsigned)a.count), dim3(block), lds, s, a);
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
