// Host side of the penalty mode (section 2.2, the prior method): per sweep,
// the threshold table for the current mu, two checkerboard half-sweeps, the
// charge read back, and the controller step mu += kappa (Q - sum S) / N, all
// in the same FP64 expressions the method's definition gives.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "../../include/lattice.h"
#include "internal.h"
#include "kernels.h"

using namespace lat;
using namespace lat::detail;

namespace {

void build_mu_table(double Delta, double V, double J, double T, double mu, std::vector<uint32_t> &tab)
{
    tab.assign(kMuTabSize, 0u);
    for (int nD = -1; nD <= 1; ++nD)
        for (int nV = -8; nV <= 8; ++nV)
            for (int nJ = -8; nJ <= 8; ++nJ)
                for (int dS = -2; dS <= 2; ++dS) {
                    const double dE = Delta * nD + V * nV + 0.25 * J * nJ - mu * dS;
                    uint32_t t;
                    if (dE <= 0.0) {
                        t = 0xFFFFFFFFu;
                    } else {
                        const double f = std::floor(std::exp(-dE / T) * 4294967296.0);
                        t = f >= 4294967294.0 ? 0xFFFFFFFEu : (uint32_t)f;
                    }
                    tab[(size_t)(((nD + 1) * 17 + (nV + 8)) * 17 + (nJ + 8)) * 5 + (size_t)(dS + 2)] = t;
                }
}

}  // namespace

extern "C" {

int lattice_mu_sweeps(lattice *h, uint64_t first_sweep, uint32_t n_sweeps, double kappa, double *mu,
                      double *mu_series, int64_t *sumS_series)
{
    return guarded("lattice_mu_sweeps", [&]() -> int {
        if (!live(h)) return fail(LAT_ESTATE, "null or destroyed handle");
        if (!mu || !std::isfinite(*mu) || !std::isfinite(kappa)) return fail(LAT_EINVAL, "mu and kappa must be finite");
        if (h->enc != LAT_ENC_INT8) return fail(LAT_EINVAL, "the penalty mode takes int8 lattices");
        std::vector<uint32_t> tab;
        MuArgs a{};
        a.state = (int8_t *)h->d_state;
        a.tab = (const uint32_t *)(h->d_scratch + kScrMuTab);
        a.track = (unsigned long long *)(h->d_scratch + kScrSlots);
        a.L = h->L;
        a.key0 = (uint32_t)h->seed;
        a.key1 = (uint32_t)(h->seed >> 32);
        for (uint32_t i = 0; i < n_sweeps; ++i) {
            const uint64_t s = first_sweep + i;
            build_mu_table(h->Delta, h->V, h->J, h->T, *mu, tab);
            hipError_t e = hipMemcpyAsync(h->d_scratch + kScrMuTab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice,
                                          h->stream);
            a.s_lo = (uint32_t)s;
            a.s_hi = (uint32_t)(s >> 32);
            for (int c = 0; c < 2 && e == hipSuccess; ++c) {
                a.colour = c;
                e = launch_mu_half(a, h->stream);
            }
            if (e == hipSuccess) e = launch_observables(h->d_scratch, h->d_state, h->L, h->enc, h->stream);
            int64_t sumS = 0;
            if (e == hipSuccess)
                e = hipMemcpyAsync(&sumS, h->d_scratch + kScrObs, sizeof(sumS), hipMemcpyDeviceToHost, h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // also keeps `tab` alive for its copy
            if (e != hipSuccess) return hip_fail(e, "lattice_mu_sweeps");
            if (mu_series) mu_series[i] = *mu;
            if (sumS_series) sumS_series[i] = sumS;
            *mu = *mu + kappa * (double)(h->Q - sumS) / (double)h->N;
        }
        return LAT_OK;
    });
}

}  // extern "C"
