// gfx950 kernels of the coupled-pair Metropolis sweep (arXiv:2301.11735,
// section 3.1 update, section 3.2 parallel form) and of the observable
// reduction.  Integer-only: no floating point, no matrix cores.
//
// One phase updates the N/8 pairs a = (x, y), x = p (mod 4), y even, with
// partners b = a + D.  No updated site neighbours another updated site, so
// every pair reads only sites nobody writes in the phase and the pairs are
// independent; the phase equals their sequential composition.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "philox.h"

namespace lat {
namespace {

// S and sigma of a site code: 0 -> (0,+1), 1 -> (0,-1), 2 -> (+1,0), 3 -> (-1,0).
__device__ __forceinline__ int charge_of(uint32_t c) { return (c & 2u) ? 1 - 2 * (int)(c & 1u) : 0; }
__device__ __forceinline__ int spin_of(uint32_t c) { return (c & 2u) ? 0 : 1 - 2 * (int)(c & 1u); }

// Same-charge pair sets of section 3.1 in the paper's listing order, one
// 4-bit entry per configuration (code_a | code_b << 2), entry j at bits 4j:
//   q=+1: (2,0) (2,1) (0,2) (1,2)
//   q= 0: (2,3) (3,2) (0,0) (1,1) (0,1) (1,0)
//   q=-1: (3,0) (3,1) (0,3) (1,3)
constexpr uint32_t kSetPlus1 = 0x9862u;
constexpr uint32_t kSetZero = 0x1450BEu;
constexpr uint32_t kSetMinus1 = 0xDC73u;

// Coupled-pair Metropolis step (section 3.1) for codes (ca, cb) whose
// neighbour sums are (sSa, sGa) and (sSb, sGb).  uc picks the configuration,
// ua is the acceptance draw.  Returns the new codes through na, nb and adds
// the accepted energy-change triple to (tD, tV, tJ).
__device__ __forceinline__ void pair_move(uint32_t ca, uint32_t cb, int sSa, int sGa, int sSb, int sGb,
                                          uint32_t uc, uint32_t ua, const uint32_t *__restrict__ thr,
                                          uint32_t &na, uint32_t &nb, int &tD, int &tV, int &tJ)
{
    na = ca;
    nb = cb;
    const int Sa = charge_of(ca), Sb = charge_of(cb);
    const int q = Sa + Sb;
    if (q == 2 || q == -2) return;  // frozen pair
    const uint32_t kq = (q == 0) ? 6u : 4u;
    const uint32_t j = ((uc >> 8) * kq) >> 24;
    const uint32_t set = (q == 1) ? kSetPlus1 : ((q == 0) ? kSetZero : kSetMinus1);
    const uint32_t e = (set >> (4u * j)) & 15u;
    const uint32_t a1 = e & 3u, b1 = e >> 2;
    const int Sa1 = charge_of(a1), Sb1 = charge_of(b1);
    const int nD = Sa1 * Sa1 + Sb1 * Sb1 - Sa * Sa - Sb * Sb;
    const int nV = (Sa1 - Sa) * sSa + (Sb1 - Sb) * sSb;
    const int nJ = (spin_of(a1) - spin_of(ca)) * sGa + (spin_of(b1) - spin_of(cb)) * sGb;
    const uint32_t t = thr[(nD + 2) * (kTabV * kTabJ) + (nV + 16) * kTabJ + (nJ + 16)];
    if (t == 0xFFFFFFFFu || ua < t) {
        na = a1;
        nb = b1;
        tD += nD;
        tV += nV;
        tJ += nJ;
    }
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
__global__ void __launch_bounds__(256) k_phase_int8(PhaseArgs a)
{
    const int L = a.L, Lq = L >> 2;
    const uint32_t n_calls = (uint32_t)L * (uint32_t)L / 16u;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    int tr[3] = {0, 0, 0};
    if (t < n_calls) {
        int8_t *st = (int8_t *)a.state;
        const u32x4 w = philox4x32_10(a.s_lo, (uint32_t)a.p, t, a.s_hi, a.key0, a.key1);
        const int Dx = a.r + 4 * a.m, Dy = 1 + 2 * a.k;
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
            const uint32_t n0 = st[(size_t)y * L + xl], n1 = st[(size_t)y * L + xr];
            const uint32_t n2 = st[(size_t)yu * L + x], n3 = st[(size_t)yd * L + x];
            const uint32_t m0 = st[(size_t)yb * L + xbl], m1 = st[(size_t)yb * L + xbr];
            const uint32_t m2 = st[(size_t)ybu * L + xb], m3 = st[(size_t)ybd * L + xb];
            const int sSa = charge_of(n0) + charge_of(n1) + charge_of(n2) + charge_of(n3);
            const int sGa = spin_of(n0) + spin_of(n1) + spin_of(n2) + spin_of(n3);
            const int sSb = charge_of(m0) + charge_of(m1) + charge_of(m2) + charge_of(m3);
            const int sGb = spin_of(m0) + spin_of(m1) + spin_of(m2) + spin_of(m3);
            uint32_t na, nb;
            pair_move(ca, cb, sSa, sGa, sSb, sGb, h ? w.z : w.x, h ? w.w : w.y, a.thr, na, nb, tr[0], tr[1],
                      tr[2]);
            if (na != ca) st[ia] = (int8_t)na;
            if (nb != cb) st[ib] = (int8_t)nb;
        }
    }
    block_reduce_add<3>(tr, a.track);
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

// 16 sites of a class row starting at class position xs (periodic).
__device__ __forceinline__ uint32_t load16(const uint32_t *__restrict__ row, int W, int xs)
{
    const int jw = xs >> 4, sh = xs & 15;
    const uint32_t w0 = row[jw];
    const uint32_t w1 = row[jw + 1 == W ? 0 : jw + 1];
    return sh ? __builtin_amdgcn_alignbit(w1, w0, 2u * (uint32_t)sh) : w0;
}

__device__ __forceinline__ void sums_at(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, int sh, int &sS,
                                        int &sG)
{
    const uint32_t c0 = (w0 >> sh) & 3u, c1 = (w1 >> sh) & 3u, c2 = (w2 >> sh) & 3u, c3 = (w3 >> sh) & 3u;
    sS = charge_of(c0) + charge_of(c1) + charge_of(c2) + charge_of(c3);
    sG = spin_of(c0) + spin_of(c1) + spin_of(c2) + spin_of(c3);
}

__global__ void __launch_bounds__(1024) k_phase_2bit(PhaseArgs a)
{
    extern __shared__ uint32_t xch[];
    const int L = a.L, W = L >> 6, H = L >> 1, Lq = L >> 2;
    const int rows_per_block = blockDim.x / W;
    const int rr = threadIdx.x / W, j = threadIdx.x - rr * W;
    const int Y = blockIdx.x * rows_per_block + rr;
    uint32_t *st = (uint32_t *)a.state;
    const size_t csz = (size_t)H * W;
    const int p = a.p;
    const int pb = (p + a.r) & 3, carry = (p + a.r) >> 2;
    int dX = a.m + carry;
    if (dX >= Lq) dX -= Lq;
    int Yb = Y + a.k;
    if (Yb >= H) Yb -= H;
    int Xb = 16 * j + dX;
    if (Xb >= Lq) Xb -= Lq;

    // a side: class (p, 0) row Y word j and its four neighbour words
    uint32_t *rowA = st + (size_t)p * csz + (size_t)Y * W;
    const uint32_t A0 = rowA[j];
    const uint32_t AL = p > 0 ? st[(size_t)(p - 1) * csz + (size_t)Y * W + j]
                              : load16(st + 3 * csz + (size_t)Y * W, W, 16 * j == 0 ? Lq - 1 : 16 * j - 1);
    const uint32_t AR = p < 3 ? st[(size_t)(p + 1) * csz + (size_t)Y * W + j]
                              : load16(st + (size_t)Y * W, W, 16 * j + 1 == Lq ? 0 : 16 * j + 1);
    const uint32_t AU = st[(size_t)(4 + p) * csz + (size_t)(Y == 0 ? H - 1 : Y - 1) * W + j];
    const uint32_t AD = st[(size_t)(4 + p) * csz + (size_t)Y * W + j];
    // b side: class (pb, 1) row Yb from class position Xb, and neighbours
    uint32_t *rowB = st + (size_t)(4 + pb) * csz + (size_t)Yb * W;
    const uint32_t B0 = load16(rowB, W, Xb);
    const uint32_t BL = pb > 0 ? load16(st + (size_t)(4 + pb - 1) * csz + (size_t)Yb * W, W, Xb)
                               : load16(st + 7 * csz + (size_t)Yb * W, W, Xb == 0 ? Lq - 1 : Xb - 1);
    const uint32_t BR = pb < 3 ? load16(st + (size_t)(4 + pb + 1) * csz + (size_t)Yb * W, W, Xb)
                               : load16(st + 4 * csz + (size_t)Yb * W, W, Xb + 1 == Lq ? 0 : Xb + 1);
    const uint32_t BU = load16(st + (size_t)pb * csz + (size_t)Yb * W, W, Xb);
    const uint32_t BD = load16(st + (size_t)pb * csz + (size_t)(Yb + 1 == H ? 0 : Yb + 1) * W, W, Xb);

    int tr[3] = {0, 0, 0};
    uint32_t Anew = A0, Bnew = B0;
    const uint32_t call0 = (uint32_t)Y * (uint32_t)(Lq >> 1) + 8u * (uint32_t)j;
    for (int c = 0; c < 8; ++c) {
        const u32x4 w = philox4x32_10(a.s_lo, (uint32_t)p, call0 + (uint32_t)c, a.s_hi, a.key0, a.key1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int sh = 2 * (2 * c + h);
            const uint32_t ca = (A0 >> sh) & 3u, cb = (B0 >> sh) & 3u;
            int sSa, sGa, sSb, sGb;
            sums_at(AL, AR, AU, AD, sh, sSa, sGa);
            sums_at(BL, BR, BU, BD, sh, sSb, sGb);
            uint32_t na, nb;
            pair_move(ca, cb, sSa, sGa, sSb, sGb, h ? w.z : w.x, h ? w.w : w.y, a.thr, na, nb, tr[0], tr[1],
                      tr[2]);
            Anew ^= (na ^ ca) << sh;
            Bnew ^= (nb ^ cb) << sh;
        }
    }
    rowA[j] = Anew;
    xch[threadIdx.x] = Bnew;
    __syncthreads();
    const uint32_t nxt = xch[rr * W + (j + 1 == W ? 0 : j + 1)];
    const int jb = Xb >> 4, shb = Xb & 15;
    const uint32_t word = shb ? __builtin_amdgcn_alignbit(nxt, Bnew, 32u - 2u * (uint32_t)shb) : nxt;
    rowB[jb + 1 == W ? 0 : jb + 1] = word;
    block_reduce_add<3>(tr, a.track);
}

// ---------------------------------------------------------------------------
__global__ void k_zero_i64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Observable sums: sum S, sum S^2, bonds S S, bonds sigma sigma, sum sigma,
// staggered sigma, staggered S.  Bonds (x,y)-(x+1,y) and (x,y)-(x,y+1).
__global__ void __launch_bounds__(256) k_obs_int8(const int8_t *__restrict__ st, int L,
                                                  unsigned long long *obs)
{
    long long v[7] = {0, 0, 0, 0, 0, 0, 0};
    const size_t N = (size_t)L * L;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / L), x = (int)(i - (size_t)y * L);
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
    block_reduce_add<7>(v, obs);
}

__global__ void __launch_bounds__(256) k_obs_2bit(const uint32_t *__restrict__ st, int L,
                                                  unsigned long long *obs)
{
    long long v[7] = {0, 0, 0, 0, 0, 0, 0};
    const int W = L >> 6, H = L >> 1, Lq = L >> 2;
    const size_t csz = (size_t)H * W, nwords = 8 * csz;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords;
         i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / csz);
        const size_t rem = i - (size_t)c * csz;
        const int Y = (int)(rem / W), j = (int)(rem - (size_t)Y * W);
        const int cx = c & 3, cy = c >> 2;
        const uint32_t w = st[i];
        const uint32_t wr = cx < 3 ? st[i + csz]
                                   : load16(st + (size_t)(4 * cy) * csz + (size_t)Y * W, W,
                                            16 * j + 1 == Lq ? 0 : 16 * j + 1);
        const uint32_t wd = cy == 0 ? st[i + 4 * csz]
                                    : st[(size_t)cx * csz + (size_t)(Y + 1 == H ? 0 : Y + 1) * W + j];
        const int sg = ((cx + cy) & 1) ? -1 : 1;
        int s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const uint32_t a = (w >> (2 * t)) & 3u, r = (wr >> (2 * t)) & 3u, d = (wd >> (2 * t)) & 3u;
            const int S = charge_of(a), G = spin_of(a);
            s0 += S;
            s1 += S * S;
            s2 += S * (charge_of(r) + charge_of(d));
            s3 += G * (spin_of(r) + spin_of(d));
            s4 += G;
        }
        v[0] += s0;
        v[1] += s1;
        v[2] += s2;
        v[3] += s3;
        v[4] += s4;
        v[5] += sg * s4;
        v[6] += sg * s0;
    }
    block_reduce_add<7>(v, obs);
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_phase_int8(const PhaseArgs &a, hipStream_t s)
{
    const uint32_t n_calls = (uint32_t)a.L * (uint32_t)a.L / 16u;
    const uint32_t block = 256, grid = (n_calls + block - 1) / block;
    hipLaunchKernelGGL(k_phase_int8, dim3(grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

// Rows per block: a power of two <= 32 (so it divides the L/2 = 32W rows)
// giving about 256 threads; every block holds whole class rows.
static int rows_per_block_2bit(int W)
{
    int r = 1;
    while (r < 32 && 2 * r * W <= 256) r *= 2;
    return r;
}

hipError_t launch_phase_2bit(const PhaseArgs &a, hipStream_t s)
{
    const int W = a.L >> 6, H = a.L >> 1;
    const int R = rows_per_block_2bit(W);
    const int block = R * W, grid = H / R;
    hipLaunchKernelGGL(k_phase_2bit, dim3(grid), dim3(block), (size_t)block * 4u, s, a);
    return hipGetLastError();
}

hipError_t launch_zero_i64(unsigned long long *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_i64, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_observables(const void *state, int L, int encoding, unsigned long long *obs, hipStream_t s)
{
    hipError_t e = launch_zero_i64(obs, 7, s);
    if (e != hipSuccess) return e;
    const size_t units = encoding == 0 ? (size_t)L * L : (size_t)L * L / 16;
    size_t grid = (units + 255) / 256;
    if (grid > 4096) grid = 4096;
    if (encoding == 0)
        hipLaunchKernelGGL(k_obs_int8, dim3((unsigned)grid), dim3(256), 0, s, (const int8_t *)state, L, obs);
    else
        hipLaunchKernelGGL(k_obs_2bit, dim3((unsigned)grid), dim3(256), 0, s, (const uint32_t *)state, L, obs);
    return hipGetLastError();
}

}  // namespace lat
