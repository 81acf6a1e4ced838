// gfx950 kernel of the penalty mode (arXiv:2301.11735 section 2.2): the prior
// method the paper replaces, kept to show its defect.  The energy gets
// -mu sum S, sites are updated one at a time by the Metropolis rule on a
// checkerboard (sites of one colour never neighbour each other), and the
// host adjusts mu between sweeps.  Int8 states.
//
// Thread t of a half-sweep owns Philox call t, i.e. sites k = 2t and 2t+1 of
// the colour (site k at row k / (L/2), column 2 (k mod L/2) + ((row + c) & 1)).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace lat {
namespace {

constexpr uint32_t kDomMu = 0x600u;

__device__ __forceinline__ int sigma_c(uint32_t c) { return (c & 2u) ? 0 : 1 - 2 * (int)(c & 1u); }

__device__ __forceinline__ void mu_site(int8_t *st, const uint32_t *tab, int L, int colour, uint32_t k, uint32_t uc,
                                        uint32_t ua, int (&tr)[3])
{
    const uint32_t half = (uint32_t)L >> 1;
    const uint32_t y = k / half, xh = k - y * half;
    const uint32_t x = 2u * xh + ((y + (uint32_t)colour) & 1u);
    const uint32_t row = y * (uint32_t)L;
    const uint32_t i = row + x;
    const uint32_t xr = x + 1 == (uint32_t)L ? 0 : x + 1, xl = x == 0 ? (uint32_t)L - 1 : x - 1;
    const uint32_t rd = y + 1 == (uint32_t)L ? 0 : row + (uint32_t)L;
    const uint32_t ru = y == 0 ? (uint32_t)L * ((uint32_t)L - 1) : row - (uint32_t)L;
    const uint32_t n0 = (uint32_t)st[row + xr], n1 = (uint32_t)st[row + xl], n2 = (uint32_t)st[rd + x],
                   n3 = (uint32_t)st[ru + x];
    const int sS = charge_of(n0) + charge_of(n1) + charge_of(n2) + charge_of(n3);
    const int sG = sigma_c(n0) + sigma_c(n1) + sigma_c(n2) + sigma_c(n3);
    const uint32_t c0 = (uint32_t)st[i], c1 = uc >> 30;
    const int dS = charge_of(c1) - charge_of(c0);
    const int nD = charge_of(c1) * charge_of(c1) - charge_of(c0) * charge_of(c0);
    const int nV = dS * sS;
    const int nJ = (sigma_c(c1) - sigma_c(c0)) * sG;
    const uint32_t thr = tab[(((nD + 1) * 17 + (nV + 8)) * 17 + (nJ + 8)) * 5 + (dS + 2)];
    if (min(ua, 0xFFFFFFFEu) < thr) {
        st[i] = (int8_t)c1;
        tr[0] += nD;
        tr[1] += nV;
        tr[2] += nJ;
    }
}

__global__ void __launch_bounds__(256) k_mu_half(MuArgs a)
{
    __shared__ uint32_t s_tab[kMuTabSize];
    for (int i = threadIdx.x; i < kMuTabSize; i += blockDim.x) s_tab[i] = a.tab[i];
    __syncthreads();
    const uint32_t n_sites = (uint32_t)a.L * (uint32_t)a.L / 2u;  // sites of one colour
    int tr[3] = {0, 0, 0};
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; 2u * t < n_sites; t += gridDim.x * blockDim.x) {
        const u32x4 w = philox4x32_10(a.s_lo, kDomMu + (uint32_t)a.colour, t, a.s_hi, a.key0, a.key1);
        mu_site(a.state, s_tab, a.L, a.colour, 2u * t, w.x, w.y, tr);
        if (2u * t + 1u < n_sites) mu_site(a.state, s_tab, a.L, a.colour, 2u * t + 1u, w.z, w.w, tr);
    }
    block_reduce_add<3>(tr, a.track + 3 * (size_t)blockIdx.x);
}

}  // namespace

hipError_t launch_mu_half(const MuArgs &a, hipStream_t s)
{
    const uint32_t calls = (uint32_t)a.L * (uint32_t)a.L / 4u;
    uint32_t grid = (calls + 255u) / 256u;
    if (grid > (uint32_t)kMaxSlots) grid = (uint32_t)kMaxSlots;
    hipLaunchKernelGGL(k_mu_half, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace lat
