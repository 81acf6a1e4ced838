// gfx950 observable reduction of one lattice (sum S, sum S^2, bond sums,
// magnetisations; arXiv:2301.11735 section 2.1 energy terms) and the fold of
// the per-block partial sums into the totals.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device_common.h"

namespace lat {
namespace {

__global__ void k_zero_i64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
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

// Totals of one lattice: tracker = base triple + every tracker slot;
// observables = the first n_obs observable slots.  Written to dst (tracker,
// then the 7 sums) and, with stamp, dst[10] = the lattice's next sweep index.
__global__ void __launch_bounds__(256) k_fold_sums(uint8_t *scr, int n_obs, long long *dst, int stamp)
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
    block_reduce_store<10>(t, dst);
    if (stamp && threadIdx.x == 0) dst[10] = (long long)((const LatDesc *)(scr + kScrDesc))->next_sweep;
}

}  // namespace

hipError_t launch_zero_i64(unsigned long long *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_i64, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_observables(uint8_t *scratch, const void *state, int L, int encoding, hipStream_t s,
                              long long *record)
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
    long long *dst = record ? record : (long long *)(scratch + kScrTrack);
    hipLaunchKernelGGL(k_fold_sums, dim3(1), dim3(256), 0, s, scratch, (int)grid, dst, record ? 1 : 0);
    return hipGetLastError();
}

}  // namespace lat
