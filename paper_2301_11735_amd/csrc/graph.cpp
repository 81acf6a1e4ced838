// Observation intervals of a batch, captured into a HIP graph: per interval
// the batched sweep launch(es) and the batched observable reduction into that
// interval's slot of a caller-owned device buffer.  A replay re-runs them all;
// the sweep kernels read each lattice's next sweep index from its device
// descriptor and advance it, so consecutive replays continue the chains
// exactly as eager calls would.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/lattice.h"
#include "internal.h"
#include "kernels.h"

using namespace lat;
using namespace lat::detail;

namespace {
constexpr uint32_t kGraphMagic = 0x47524150u;
}

struct lat_batch_graph {
    std::vector<lattice *> hs;
    uint32_t sweeps = 0, intervals = 0;
    void *d_out = nullptr;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t magic = 0;
};

namespace {

bool graph_live(const lat_batch_graph *g) { return g != nullptr && g->magic == kGraphMagic; }

void release(lat_batch_graph *g)
{
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->magic = 0;
    delete g;
}

}  // namespace

extern "C" {

int lattice_batch_graph_create(lattice *const *hs, int32_t count, uint32_t sweeps, uint32_t intervals, void *d_out,
                               size_t out_bytes, void *hip_stream, lat_batch_graph **out)
{
    return guarded("lattice_batch_graph_create", [&]() -> int {
        if (!out) return fail(LAT_EINVAL, "null output handle");
        *out = nullptr;
        if (count <= 0 || !hs || !d_out || sweeps == 0 || intervals == 0) return fail(LAT_EINVAL, "bad batch graph arguments");
        if (out_bytes / 80u / (size_t)count < (size_t)intervals)
            return fail(LAT_ENOMEM, "output buffer smaller than 80 bytes per lattice and interval");
        for (int32_t i = 0; i < count; ++i) {
            if (!live(hs[i])) return fail(LAT_ESTATE, "null or destroyed handle in batch");
            if (hs[i]->path == kPathPhase)
                return fail(LAT_EINVAL, "a batch graph takes lattices on the on-chip or the multi-block word path "
                                        "(L <= 2048 with L % 64 == 0, or L <= 512)");
        }
        {
            std::vector<const lattice *> seen(hs, hs + count);
            std::sort(seen.begin(), seen.end());
            if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
                return fail(LAT_EINVAL, "a lattice appears twice in the batch");
        }

        auto *g = new lat_batch_graph();
        g->hs.assign(hs, hs + count);
        g->sweeps = sweeps;
        g->intervals = intervals;
        g->d_out = d_out;
        g->stream = (hipStream_t)hip_stream;

        // Capture on a private stream (the caller's may be the null stream, which
        // cannot be captured); nothing runs until a replay.
        hipStream_t cs = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) {
            release(g);
            return hip_fail(e, "capture stream");
        }
        std::vector<uint64_t> done(g->hs.size());
        for (size_t i = 0; i < g->hs.size(); ++i) done[i] = g->hs[i]->done;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
        int rc = LAT_OK;
        if (e == hipSuccess) {
            std::vector<lattice *> small, big;
            for (lattice *h : g->hs) (h->path == kPathLds ? small : big).push_back(h);
            for (uint32_t k = 0; k < intervals && rc == LAT_OK; ++k) {
                unsigned long long *slot = (unsigned long long *)d_out + 10 * (size_t)count * k;
                if (big.empty()) {
                    // the sweeps and the interval's observables, in one launch for the word form
                    rc = enqueue_lds_sweeps(g->hs.data(), count, nullptr, sweeps, cs, /*tune=*/false, slot);
                } else {
                    // the multi-block word path computes its schedules on the
                    // device, so its launch series replays like the on-chip
                    // one; one launch per phase, since a graph's kernel node
                    // does not guarantee the co-residency that the persistent
                    // form's device-wide barrier needs
                    rc = enqueue_lds_sweeps(small.data(), (int32_t)small.size(), nullptr, sweeps, cs, false);
                    if (rc == LAT_OK)
                        rc = enqueue_offchip_sweeps(big.data(), (int32_t)big.size(), nullptr, sweeps, cs,
                                                    /*convert=*/true, /*persistent=*/false);
                    if (rc == LAT_OK) rc = enqueue_observables_batch(g->hs.data(), count, slot, cs);
                }
            }
            const hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
            if (rc == LAT_OK && e2 != hipSuccess) e = e2;
        }
        // the capture advanced the host-side sweep counters; nothing has run yet
        for (size_t i = 0; i < g->hs.size(); ++i) g->hs[i]->done = done[i];
        if (e == hipSuccess && rc == LAT_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cs);
        if (rc != LAT_OK) {
            release(g);
            return rc;
        }
        if (e != hipSuccess) {
            release(g);
            return hip_fail(e, "batch graph capture");
        }
        g->magic = kGraphMagic;
        *out = g;
        return LAT_OK;
    });
}

int lattice_batch_graph_launch(lat_batch_graph *g, uint32_t times)
{
    return guarded("lattice_batch_graph_launch", [&]() -> int {
        if (!graph_live(g)) return fail(LAT_ESTATE, "null or destroyed batch graph");
        for (uint32_t t = 0; t < times; ++t) {
            const hipError_t e = hipGraphLaunch(g->exec, g->stream);
            if (e != hipSuccess) return hip_fail(e, "batch graph launch");
            for (lattice *h : g->hs) h->done += (uint64_t)g->sweeps * g->intervals;
        }
        return LAT_OK;
    });
}

int lattice_batch_graph_read(lat_batch_graph *g, lat_obs *out)
{
    return guarded("lattice_batch_graph_read", [&]() -> int {
        if (!graph_live(g)) return fail(LAT_ESTATE, "null or destroyed batch graph");
        if (!out) return fail(LAT_EINVAL, "null output");
        const size_t n = g->hs.size();
        std::vector<int64_t> v(n * 10 * g->intervals);
        hipError_t e = hipMemcpyAsync(v.data(), g->d_out, v.size() * 8, hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) return hip_fail(e, "lattice_batch_graph_read");
        for (uint32_t k = 0; k < g->intervals; ++k)
            for (size_t i = 0; i < n; ++i) {
                lat_obs &o = out[k * n + i];
                fill_obs(g->hs[i], &v[10 * (k * n + i)], &o);
                o.sweep -= (uint64_t)g->sweeps * (g->intervals - 1u - k);
            }
        return LAT_OK;
    });
}

int lattice_batch_graph_destroy(lat_batch_graph *g)
{
    return guarded("lattice_batch_graph_destroy", [&]() -> int {
        if (!graph_live(g)) return fail(LAT_ESTATE, "null or destroyed batch graph");
        const hipError_t e = hipStreamSynchronize(g->stream);
        release(g);
        return e == hipSuccess ? LAT_OK : hip_fail(e, "lattice_batch_graph_destroy");
    });
}

}  // extern "C"
