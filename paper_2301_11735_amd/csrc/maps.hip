// gfx950 kernel of the map mode (arXiv:2301.11735 section 3.2): the paper's
// random maps of non-interacting coupled pairs, built on the device.
//
// One block per lattice (up to 256 lattices per launch, L <= 256).  Per map:
//   1. the block clears a bitmap of marked sites;
//   2. wave 0 builds the map with the paper's sequential algorithm -- draw a
//      site until an unmarked one comes up, mark it; the same for the
//      partner; record the pair; mark the neighbours of both -- its 64 lanes
//      computing the next 256 site draws at once and the wave taking them in
//      draw order;
//   3. all threads apply one coupled-pair Metropolis step (section 3.1) to the
//      map's pairs in parallel.  No two pairs of a map interact, so this equals
//      applying them one after another; a pair's own sites may be neighbours,
//      and the bond between them then enters the energy change once.
// The codes (one byte per site), the bitmap, the pair list and the full
// threshold table over (nD, nV, nJ) live in LDS for all maps of the launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace lat {
namespace {

constexpr uint32_t kDomMap = 0x400u;      // site draws of a map's construction
constexpr uint32_t kDomMapStep = 0x500u;  // configuration and acceptance draws of its pairs

// Same-charge configurations of a pair (section 3.1 listing), nibble j of the
// constant for q = +1, 0, -1 holding code_a | code_b << 2.
constexpr uint32_t kSetQp1 = 0x9862u;    // (2,0) (2,1) (0,2) (1,2)
constexpr uint32_t kSetQ0 = 0x1450BEu;   // (2,3) (3,2) (0,0) (1,1) (0,1) (1,0)
constexpr uint32_t kSetQm1 = 0xDC73u;    // (3,0) (3,1) (0,3) (1,3)

__device__ __forceinline__ int sigma_of(uint32_t c) { return (c & 2u) ? 0 : 1 - 2 * (int)(c & 1u); }

__device__ __forceinline__ void site_neighbours(int L, uint32_t s, uint32_t (&nb)[4])
{
    const uint32_t y = s / (uint32_t)L, x = s - y * (uint32_t)L;
    const uint32_t row = y * (uint32_t)L;
    nb[0] = row + (x + 1 == (uint32_t)L ? 0 : x + 1);
    nb[1] = row + (x == 0 ? (uint32_t)L - 1 : x - 1);
    nb[2] = (y + 1 == (uint32_t)L ? 0 : row + (uint32_t)L) + x;
    nb[3] = (y == 0 ? (uint32_t)L * ((uint32_t)L - 1) : row - (uint32_t)L) + x;
}

// Map m into pairs[] (a | b << 16), by the calling wave (several waves of a
// block build different maps at once, each in its own bitmap).  Per round the
// 64 lanes compute the next 256 site draws, their neighbours and whether each
// was already marked when the round began (one ballot per draw slot); then the
// wave walks the draws in draw order with uniform control flow: a draw marked
// at the start of the round is rejected without touching LDS, any other is
// checked against the live bitmap (a broadcast LDS read, which the in-order LDS
// queue orders after the marks already issued).  Marks are LDS atomic ors.
template <bool NN>
__device__ void build_map(uint32_t *bitmap, uint32_t *pairs, int L, uint32_t N, uint32_t n_pairs, uint32_t m_lo,
                          uint32_t m_hi, uint32_t key0, uint32_t key1)
{
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t k = 0, count = 0, need_b = 0, a_site = 0;
    uint32_t an[4] = {0u, 0u, 0u, 0u};  // neighbours of the pending first site
    while (count < n_pairs) {
        // draws k .. k+255: draw d is word d mod 4 of Philox call d / 4, held by lane d / 4
        const u32x4 w = philox4x32_10(m_lo, kDomMap, (k >> 2) + lane, m_hi, key0, key1);
        const uint32_t raw[4] = {w.x, w.y, w.z, w.w};
        const uint32_t c[4] = {mulhi_u32(w.x, N), mulhi_u32(w.y, N), mulhi_u32(w.z, N), mulhi_u32(w.w, N)};
        uint32_t nbv[4][4];
        uint64_t pre[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            site_neighbours(L, c[q], nbv[q]);
            pre[q] = __ballot((bitmap[c[q] >> 5] >> (c[q] & 31u)) & 1u);
        }
        for (int l = 0; l < 64 && count < n_pairs; ++l) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (count >= n_pairs) continue;
                if (NN && need_b) {
                    // nearest-neighbour partner: this draw picks neighbour raw >> 30 of a
                    need_b = 0;
                    const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)raw[q], l) >> 30;
                    const uint32_t b = d == 0 ? an[0] : d == 1 ? an[1] : d == 2 ? an[2] : an[3];
                    const uint32_t bw = (uint32_t)__builtin_amdgcn_readfirstlane((int)bitmap[b >> 5]);
                    if (bw & (1u << (b & 31u))) continue;  // drop the pair, start over
                    uint32_t bn[4];
                    site_neighbours(L, b, bn);
                    if (lane == 0) {
                        pairs[count] = a_site | (b << 16);
                        atomicOr(&bitmap[a_site >> 5], 1u << (a_site & 31u));
                        atomicOr(&bitmap[b >> 5], 1u << (b & 31u));
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            atomicOr(&bitmap[an[e] >> 5], 1u << (an[e] & 31u));
                            atomicOr(&bitmap[bn[e] >> 5], 1u << (bn[e] & 31u));
                        }
                    }
                    ++count;
                    continue;
                }
                if ((pre[q] >> l) & 1u) continue;
                const uint32_t site = (uint32_t)__builtin_amdgcn_readlane((int)c[q], l);
                const uint32_t word = (uint32_t)__builtin_amdgcn_readfirstlane((int)bitmap[site >> 5]);
                if (word & (1u << (site & 31u))) continue;
                if (NN) {
                    // first site of a nearest-neighbour pair: marked only once the pair is kept
                    a_site = site;
#pragma unroll
                    for (int d = 0; d < 4; ++d) an[d] = (uint32_t)__builtin_amdgcn_readlane((int)nbv[q][d], l);
                    need_b = 1;
                    continue;
                }
                if (lane == 0) atomicOr(&bitmap[site >> 5], 1u << (site & 31u));
                if (!need_b) {
                    a_site = site;
#pragma unroll
                    for (int d = 0; d < 4; ++d) an[d] = (uint32_t)__builtin_amdgcn_readlane((int)nbv[q][d], l);
                    need_b = 1;
                } else {
                    if (lane == 0) {
                        pairs[count] = a_site | (site << 16);
#pragma unroll
                        for (int d = 0; d < 4; ++d) atomicOr(&bitmap[an[d] >> 5], 1u << (an[d] & 31u));
                    }
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)nbv[q][d], l);
                        if (lane == 0) atomicOr(&bitmap[t >> 5], 1u << (t & 31u));
                    }
                    ++count;
                    need_b = 0;
                }
            }
        }
        k += 256u;
    }
}

// Sums of S and sigma over the neighbours of s other than `other`; adj = 1 if
// `other` is one of them.
__device__ __forceinline__ void side_sum(const uint8_t *codes, int L, uint32_t s, uint32_t other, int &sS, int &sG,
                                         int &adj)
{
    uint32_t nb[4];
    site_neighbours(L, s, nb);
    sS = 0;
    sG = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        if (nb[d] == other) {
            adj = 1;
            continue;
        }
        const uint32_t c = codes[nb[d]];
        sS += charge_of(c);
        sG += sigma_of(c);
    }
}

// One coupled-pair Metropolis step on sites (a, b), a and b possibly adjacent.
__device__ __forceinline__ void map_pair_step(uint8_t *codes, const uint32_t *thr, int L, uint32_t a, uint32_t b,
                                              uint32_t uc, uint32_t ua, int (&tr)[3])
{
    const uint32_t ca = codes[a], cb = codes[b];
    const int Sa = charge_of(ca), Sb = charge_of(cb), q = Sa + Sb;
    if (q == 2 || q == -2) return;
    const uint32_t kq = q == 0 ? 6u : 4u;
    const uint32_t j = ((uc >> 8) * kq) >> 24;
    const uint32_t cfg = ((q == 1 ? kSetQp1 : q == 0 ? kSetQ0 : kSetQm1) >> (4u * j)) & 15u;
    const uint32_t na = cfg & 3u, nb = cfg >> 2;
    int sSa, sGa, sSb, sGb, adj = 0;
    side_sum(codes, L, a, b, sSa, sGa, adj);
    side_sum(codes, L, b, a, sSb, sGb, adj);
    const int Ga = sigma_of(ca), Gb = sigma_of(cb);
    const int Sna = charge_of(na), Snb = charge_of(nb), Gna = sigma_of(na), Gnb = sigma_of(nb);
    const int nD = Sna * Sna - Sa * Sa + Snb * Snb - Sb * Sb;
    const int nV = (Sna - Sa) * sSa + (Snb - Sb) * sSb + adj * (Sna * Snb - Sa * Sb);
    const int nJ = (Gna - Ga) * sGa + (Gnb - Gb) * sGb + adj * (Gna * Gnb - Ga * Gb);
    const uint32_t t = thr[(nD + 2) * (kTabV * kTabJ) + (nV + 16) * kTabJ + (nJ + 16)];
    if (min(ua, 0xFFFFFFFEu) < t) {
        codes[a] = (uint8_t)na;
        codes[b] = (uint8_t)nb;
        tr[0] += nD;
        tr[1] += nV;
        tr[2] += nJ;
    }
}

__global__ void __launch_bounds__(kMapThreads) k_map_steps(MapArgs args)
{
    extern __shared__ uint32_t smem[];
    uint8_t *scr = args.scratch[blockIdx.x];
    const LatDesc d = *(const LatDesc *)(scr + kScrDesc);
    const int L = d.L;
    const uint32_t N = (uint32_t)L * (uint32_t)L;
    const uint32_t per = args.nn ? 20u : 10u;
    const uint32_t n_pairs = N / per < 1u ? 1u : N / per;
    const uint32_t G = (uint32_t)args.builders;            // maps built at once, one per wave
    const uint32_t bwords = (N + 31u) / 32u;
    uint32_t *thr = smem;                                   // kTabSize
    uint8_t *codes = (uint8_t *)(smem + kTabSize);          // N bytes
    uint32_t *bitmaps = smem + kTabSize + (N + 3u) / 4u;    // G x bwords
    uint32_t *pairs = bitmaps + G * bwords;                 // G x n_pairs

    const uint32_t *g_thr = (const uint32_t *)(scr + kScrFullTab);
    for (uint32_t i = threadIdx.x; i < (uint32_t)kTabSize; i += blockDim.x) thr[i] = g_thr[i];
    if (d.enc == 0) {
        const uint8_t *src = (const uint8_t *)d.state;
        for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) codes[i] = src[i];
    } else {
        // 2-bit class layout: class 4*(y&1) + (x&3), (L/2) rows of L/64 words
        const uint32_t *src = (const uint32_t *)d.state;
        const uint32_t W = (uint32_t)L >> 6, csz = ((uint32_t)L >> 1) * W;
        for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) {
            const uint32_t y = i / (uint32_t)L, x = i - y * (uint32_t)L;
            const uint32_t c = 4u * (y & 1u) + (x & 3u), X = x >> 2;
            codes[i] = (uint8_t)((src[c * csz + (y >> 1) * W + (X >> 4)] >> (2u * (X & 15u))) & 3u);
        }
    }
    __syncthreads();

    int tr[3] = {0, 0, 0};
    const uint64_t first = ((uint64_t)args.first_map_hi << 32) | args.first_map_lo;
    const uint32_t wave = threadIdx.x >> 6;
    for (uint32_t m0 = 0; m0 < args.n_maps; m0 += G) {
        const uint32_t group = min(G, args.n_maps - m0);
        // maps depend only on the seed and their index: build `group` of them at once
        for (uint32_t i = threadIdx.x; i < group * bwords; i += blockDim.x) bitmaps[i] = 0u;
        __syncthreads();
        if (wave < group) {
            const uint64_t m = first + m0 + wave;
            if (args.nn)
                build_map<true>(bitmaps + wave * bwords, pairs + wave * n_pairs, L, N, n_pairs, (uint32_t)m,
                                (uint32_t)(m >> 32), d.key0, d.key1);
            else
                build_map<false>(bitmaps + wave * bwords, pairs + wave * n_pairs, L, N, n_pairs, (uint32_t)m,
                                 (uint32_t)(m >> 32), d.key0, d.key1);
        }
        __syncthreads();
        // ...then apply them in map order
        for (uint32_t g = 0; g < group; ++g) {
            const uint64_t m = first + m0 + g;
            const uint32_t m_lo = (uint32_t)m, m_hi = (uint32_t)(m >> 32);
            const uint32_t *mp = pairs + g * n_pairs;
            // pairs 2c and 2c+1 share Philox call c
            for (uint32_t c = threadIdx.x; 2u * c < n_pairs; c += blockDim.x) {
                const u32x4 w = philox4x32_10(m_lo, kDomMapStep, c, m_hi, d.key0, d.key1);
                const uint32_t p0 = mp[2u * c];
                map_pair_step(codes, thr, L, p0 & 0xFFFFu, p0 >> 16, w.x, w.y, tr);
                if (2u * c + 1u < n_pairs) {
                    const uint32_t p1 = mp[2u * c + 1u];
                    map_pair_step(codes, thr, L, p1 & 0xFFFFu, p1 >> 16, w.z, w.w, tr);
                }
            }
            __syncthreads();
        }
    }

    if (d.enc == 0) {
        uint8_t *dst = (uint8_t *)d.state;
        for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) dst[i] = codes[i];
    } else {
        uint32_t *dst = (uint32_t *)d.state;
        const uint32_t W = (uint32_t)L >> 6, H = (uint32_t)L >> 1, csz = H * W;
        for (uint32_t i = threadIdx.x; i < 8u * csz; i += blockDim.x) {
            const uint32_t c = i / csz, rem = i - c * csz, Y = rem / W, jw = rem - Y * W;
            const uint32_t y = 2u * Y + (c >> 2), x0 = c & 3u;
            uint32_t v = 0;
            for (uint32_t t = 0; t < 16u; ++t) v |= (uint32_t)codes[y * (uint32_t)L + 4u * (16u * jw + t) + x0] << (2u * t);
            dst[i] = v;
        }
    }
    block_reduce_add<3>(tr, (unsigned long long *)(scr + kScrTrackBase));
}

}  // namespace

hipError_t launch_map_steps(const MapArgs &a, int max_L, hipStream_t s)
{
    // as many concurrent builders (at most one per wave) as LDS allows
    MapArgs b = a;
    b.builders = 1;
    for (int g = kMapThreads / 64; g > 1; g /= 2)
        if (map_lds_bytes(max_L, g) <= kMapLdsMax) {
            b.builders = g;
            break;
        }
    hipLaunchKernelGGL(k_map_steps, dim3((unsigned)b.count), dim3(kMapThreads), map_lds_bytes(max_L, b.builders), s,
                       b);
    return hipGetLastError();
}

hipError_t init_map_kernel_attributes()
{
    return hipFuncSetAttribute((const void *)k_map_steps, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kMapLdsMax);
}

}  // namespace lat
