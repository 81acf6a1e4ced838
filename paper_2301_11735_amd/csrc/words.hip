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

#include "device_common.h"
#include "word_task.h"

namespace lat {
namespace {

template <int Q>
__global__ void __launch_bounds__(kWordsThreads) k_phase_words(WordsArgs a)
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
        for (int i = threadIdx.x; i < kDevTabEntries; i += kWordsThreads) s_tab[i] = g_tab[i];
        for (int i = threadIdx.x; i < kTransEntries; i += kWordsThreads) s_transd[i] = g_transd[i];
    }
    const uint64_t s = d.next_sweep + a.iter;
    int r, mm[4], kk[4];
    device_schedule(d.L, d.key0, d.key1, s, r, mm, kk);
    const int p = a.p;
    WordPhase f;
    f.W = d.L >> 6;
    f.H = d.L >> 1;
    f.Lq = d.L >> 2;
    f.magicW = f.W == 1 ? 0u : (uint32_t)((0x100000000ull + (uint64_t)f.W - 1u) / (uint64_t)f.W);
    f.key0 = d.key0;
    f.key1 = d.key1;
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
    __syncthreads();

    const uint32_t b = blockIdx.x - a.first_block[li];
    const uint32_t task = b * kWordsThreads + threadIdx.x;
    int tr[3] = {0, 0, 0};
    // tasks = Q * csz is a multiple of Q, so a word's lanes are all in or all out
    if (task < (uint32_t)Q * csz) word_task<Q, false, false, true>(st, f, task, s_tab, s_transd, tr);
    block_reduce_add<3>(tr, (unsigned long long *)(scr + kScrSlots) + 3 * (size_t)b);
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

int words_lanes(int L)
{
    if (L <= 512) return 8;
    if (L <= 1024) return 4;
    if (L <= 2048) return 2;
    return 1;
}

hipError_t launch_phase_words(const WordsArgs &a, int Q, hipStream_t s)
{
    const dim3 grid(a.first_block[a.count]), block(kWordsThreads);
    switch (Q) {
    case 1: hipLaunchKernelGGL(k_phase_words<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_phase_words<2>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_phase_words<4>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(k_phase_words<8>, grid, block, 0, s, a); break;
    }
    return hipGetLastError();
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
