// gfx950 phase kernels of the coupled-pair Metropolis sweep on one lattice
// (arXiv:2301.11735, section 3.1 update, section 3.2 parallel form): one
// launch per phase, or all phases of a call in one cooperative launch.
// Integer-only: no floating point, no matrix cores.
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

#include "device_common.h"

namespace lat {
namespace {

// ---------------------------------------------------------------------------
// int8 layout: one code per byte, row-major.  Thread t owns Philox call t,
// i.e. pairs 2t and 2t+1 (words 0,1 and 2,3 of the call).
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

// MinWaves > 1 asks the compiler to fit MinWaves waves per SIMD (at most
// 512/MinWaves VGPRs), e.g. two 1024-thread blocks per compute unit at 8.
// The ten words one thread reads for its 16 pairs: its a-word, the a-words'
// left/right/up/down neighbour words, and the same five for the 16 partners
// (the b-side words start mid-word and are funnel-shifted into place).
// Seven of them start mid-word (by the same shift for every thread of a
// phase): both words covering each are fetched, and the funnel shift into
// place waits until the group is computed, so a prefetch never waits for its
// own loads.
struct PairWords {
    uint32_t A0, AU, AD;
    uint32_t ALlo, ALhi, ARlo, ARhi, B0lo, B0hi, BLlo, BLhi, BRlo, BRhi, BUlo, BUhi, BDlo, BDhi;
};

// LDS tables of the 2-bit phase kernels, in 8-byte units: the device
// threshold table, one pad entry, the delta transition table (16-byte
// aligned), and two spare entries that absorb the writes of threads past the
// end during staging.  Staging moves 16 bytes (two units) at a time.
constexpr int kLdsTransD = kDevTabEntries + 1;                // 934: 16-byte aligned
constexpr int kLdsTabUnits = kLdsTransD + 2 * kTransEntries;  // 1126
constexpr int kLdsTabPairs = kLdsTabUnits / 2;                // 563
static_assert((kLdsTransD * 8) % 16 == 0 && kLdsTabUnits % 2 == 0, "delta table alignment");
static_assert(kScrTrans >= (size_t)kLdsTransD * 8, "the last device-table pair reads scratch, not past it");

// Units 2i and 2i+1 of the LDS tables from the lattice's scratch.  The pair
// holding the pad unit reads the scratch bytes after the device table.
__device__ __forceinline__ uint4 table_pair(const PhaseArgs &a, int i)
{
    return 2 * i < kLdsTransD ? *(const uint4 *)(a.dev_tab + 2 * i) : a.trans_d[i - kLdsTransD / 2];
}

// One phase of the 2-bit lattice by this block: row groups blockIdx.x,
// blockIdx.x + gridDim.x, ...
//
// s_tabs holds kLdsTabUnits + 2 entries.  Stage false: the tables are
// already there.  Stage true: they are copied here; the table loads are
// issued first, then the first group's words, so that the LDS writes wait
// only for the former and the word loads overlap the staging.
template <bool Stage>
__device__ __forceinline__ void phase_2bit(const PhaseArgs &a, int rows_per_block, uint2 *s_tabs, uint32_t *xch,
                                           int (&tr)[3])
{
    const uint2 *s_tab = s_tabs;
    const uint4 *s_transd = (const uint4 *)(s_tabs + kLdsTransD);
    const int L = a.L, W = L >> 6, H = L >> 1, Lq = L >> 2;
    const int rr = W == 1 ? (int)threadIdx.x : (int)__umulhi(threadIdx.x, a.magicW), j = (int)threadIdx.x - rr * W;
    const int n_groups = H >> __builtin_ctz((unsigned)rows_per_block);  // a power of two
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
        w.A0 = word_at(st, oA0 + ro + j);
        w.AU = word_at(st, oAV + roU + j);
        w.AD = word_at(st, oAV + ro + j);
        load_pair(st, oAL + ro, W, xAL, w.ALlo, w.ALhi);
        load_pair(st, oAR + ro, W, xAR, w.ARlo, w.ARhi);
        load_pair(st, oB0 + rob, W, Xb, w.B0lo, w.B0hi);
        load_pair(st, oBL + rob, W, xBL, w.BLlo, w.BLhi);
        load_pair(st, oBR + rob, W, xBR, w.BRlo, w.BRhi);
        load_pair(st, oBV + rob, W, Xb, w.BUlo, w.BUhi);
        load_pair(st, oBV + robD, W, Xb, w.BDlo, w.BDhi);
        return w;
    };
    // funnel shifts (uniform per phase: 2 * (x mod 16) for each start x)
    const uint32_t fAL = 2u * (uint32_t)(xAL & 15), fAR = 2u * (uint32_t)(xAR & 15);
    const uint32_t fB = 2u * (uint32_t)(Xb & 15), fBL = 2u * (uint32_t)(xBL & 15), fBR = 2u * (uint32_t)(xBR & 15);

    // Draws of the group's 8 Philox calls (call c serves pairs 2c and 2c+1).
    auto call_of = [&](int gg, int c) {
        const uint32_t call0 = (uint32_t)row_of(gg) * (uint32_t)(Lq >> 1) + 8u * (uint32_t)j;
        return philox4x32_10(a.s_lo, (uint32_t)p, call0 + (uint32_t)c, a.s_hi, a.key0, a.key1);
    };
    // Updates the 16 pairs of group gg from its words cw.
    auto group = [&](const PairWords &cw, int gg, int bb) {
        const int Y = row_of(gg), Yb = brow_of(Y);
        const uint32_t B0 = __builtin_amdgcn_alignbit(cw.B0hi, cw.B0lo, fB);
        const SideSums sa = side_sums(__builtin_amdgcn_alignbit(cw.ALhi, cw.ALlo, fAL),
                                      __builtin_amdgcn_alignbit(cw.ARhi, cw.ARlo, fAR), cw.AU, cw.AD);
        const SideSums sb = side_sums(__builtin_amdgcn_alignbit(cw.BLhi, cw.BLlo, fBL),
                                      __builtin_amdgcn_alignbit(cw.BRhi, cw.BRlo, fBR),
                                      __builtin_amdgcn_alignbit(cw.BUhi, cw.BUlo, fB),
                                      __builtin_amdgcn_alignbit(cw.BDhi, cw.BDlo, fB));
        // bpack of site t = (sumS_a+4, sumS_b+4, sumsig_a+4, sumsig_b+4): site
        // t = 4k + g is byte k of nibble plane g (g = 0, 2: even sites, low and
        // high nibbles; g = 1, 3: odd sites).  Philox call c serves t = 2c and
        // 2c+1, so calls 0,2,4,6 need planes 0 and 1, calls 1,3,5,7 planes 2
        // and 3; handling them in that order keeps 8 packed words live.
        uint32_t dlo = 0u, dhi = 0u, packed = 0u;  // code changes of pairs 0-7 and 8-15
        const uint32_t kq2w = word_kq2(cw.A0, B0);
        const uint32_t st8[2] = {pair_states8(cw.A0, B0, 0), pair_states8(cw.A0, B0, 1)};
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
                const u32x4 w = call_of(gg, c);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int t = 2 * c + h;
                    const uint32_t s0 = (st8[t >> 3] >> (4 * (t & 7))) & 15u;
                    const uint32_t fields = 0x00030003u << (2 * (t & 7));
                    pair_step_delta(s0, (kq2w >> (2 * t)) & 3u, h ? go[k] : ge[k], h ? w.z : w.x, h ? w.w : w.y,
                                    s_transd, s_tab, fields, packed, t < 8 ? dlo : dhi);
                }
            }
        }
        unpack_tracker(packed, tr);
        const uint32_t Anew = cw.A0 ^ __builtin_amdgcn_perm(dhi, dlo, 0x05040100u);
        const uint32_t Bnew = B0 ^ __builtin_amdgcn_perm(dhi, dlo, 0x07060302u);
        word_put(st, oA0 + (uint32_t)Y * W + j, Anew);
        uint32_t *x = xch + bb * blockDim.x;
        x[threadIdx.x] = Bnew;
        __syncthreads();
        const uint32_t nb = x[rr * W + j_next];
        const uint32_t word = shb ? __builtin_amdgcn_alignbit(nb, Bnew, 32u - 2u * (uint32_t)shb) : nb;
        word_put(st, oB0 + (uint32_t)Yb * W + jw_out, word);
    };

    // Each group's words are fetched before the previous group is computed.
    // Every word read is either never written in this phase or written only
    // by this block in the iteration that owns it, after its read.
    int g = blockIdx.x;
    PairWords cur;  // loaded before it is read
    if (Stage) {
        constexpr int kTot = kLdsTabPairs, kK = 2;  // two 16-byte loads a thread cover 512-thread blocks
        const int bd = rows_per_block * W;  // the block size of every launch of this form
        uint4 sv[kK];
        int si[kK];
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            si[k] = min((int)threadIdx.x + k * bd, kTot);
            sv[k] = table_pair(a, min(si[k], kTot - 1));
        }
        // unconditional (clamped) and kept after the table loads, so that
        // the LDS writes below wait for the table loads only; the loop skips
        // a block without a group
        __builtin_amdgcn_sched_barrier(0);
        cur = load_words(min(g, n_groups - 1));
        uint4 *s_pairs = (uint4 *)s_tabs;
#pragma unroll
        for (int k = 0; k < kK; ++k) s_pairs[si[k]] = sv[k];
        for (int i = (int)threadIdx.x + kK * bd; i < kTot; i += bd) s_pairs[i] = table_pair(a, i);
        __syncthreads();
    } else if (g < n_groups) {
        cur = load_words(g);
    }
    int buf = 0;
    for (; g < n_groups; g += gridDim.x, buf ^= 1) {
        const int gn = g + gridDim.x;
        PairWords nxt;  // read only when loaded
        if (gn < n_groups) nxt = load_words(gn);
        group(cur, g, buf);
        cur = nxt;
    }
    __syncthreads();  // the exchange buffer is reused by the next phase
}

template <int MinWaves>
__global__ void __launch_bounds__(1024, MinWaves) k_phase_2bit(PhaseArgs a, int rows_per_block)
{
    __shared__ __align__(16) uint2 s_tabs[kLdsTabUnits + 2];
    extern __shared__ uint32_t xch[];  // 2 x blockDim (double buffered)
    int tr[3] = {0, 0, 0};
    phase_2bit<true>(a, rows_per_block, s_tabs, xch, tr);
    block_reduce_add<3>(tr, a.track + 3 * (size_t)blockIdx.x);
}

// Persistent form: `sweeps` sweeps from sweep a.s_lo|a.s_hi in one launch of
// co-resident blocks (cooperative launch), tables staged once, schedules
// computed on the device, a device-wide barrier after every phase.
template <int MinWaves>
__global__ void __launch_bounds__(1024, MinWaves) k_sweeps_2bit(PhaseArgs a, int rows_per_block, uint32_t sweeps,
                                                                unsigned *counter, unsigned *err)
{
    __shared__ __align__(16) uint2 s_tabs[kLdsTabUnits + 2];
    extern __shared__ uint32_t xch[];
    for (int i = threadIdx.x; i < kLdsTabPairs; i += blockDim.x) ((uint4 *)s_tabs)[i] = table_pair(a, i);
    __syncthreads();
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
            phase_2bit<false>(b, rows_per_block, s_tabs, xch, tr);
            arrivals += gridDim.x;
            grid_barrier(counter, arrivals, err);
        }
    }
    block_reduce_add<3>(tr, a.track + 3 * (size_t)blockIdx.x);
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
// by default the largest giving at most max_threads threads.  Every block
// holds whole class rows.  For one launch per phase the default is blocks of
// at most 512 threads, two per compute unit (16 waves, as one 1024-thread
// block): measured 1.5% faster than one 1024-thread block at L = 8192.
static int rows_per_block_2bit(int W, int requested, int max_threads)
{
    const int cap = requested > 0 ? requested : 32;
    int r = 1;
    while (r < 32 && 2 * r <= cap && 2 * r * W <= max_threads) r *= 2;
    return r;
}

hipError_t launch_phase_2bit(const PhaseArgs &a, const Tuning2Bit &t, hipStream_t s)
{
    const int W = a.L >> 6, H = a.L >> 1;
    const int R = rows_per_block_2bit(W, t.rows_per_block, t.rows_per_block > 0 ? 1024 : 512);
    const int block = R * W;
    int grid = H / R;
    const int bpc = t.blocks_per_cu > 0 ? t.blocks_per_cu : 2;
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
    const int W = L >> 6, R = rows_per_block_2bit(W, t.rows_per_block, 1024), block = R * W;
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


}  // namespace lat
