// Host side of the map mode (section 3.2 random maps of non-interacting
// coupled pairs): argument checks and the batched launch.  Map construction
// and the pair updates run in the kernel of maps.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/lattice.h"
#include "internal.h"
#include "kernels.h"

using namespace lat;
using namespace lat::detail;

namespace {

int enqueue_map_steps(lattice *const *hs, int32_t count, uint64_t first_map, uint32_t n_maps, int32_t partner,
                      hipStream_t stream)
{
    for (int32_t b = 0; b < count; b += kMaxBatch) {
        MapArgs a{};
        a.count = std::min<int32_t>(kMaxBatch, count - b);
        a.first_map_lo = (uint32_t)first_map;
        a.first_map_hi = (uint32_t)(first_map >> 32);
        a.n_maps = n_maps;
        a.nn = partner;
        int max_L = 0;
        for (int i = 0; i < a.count; ++i) {
            a.scratch[i] = hs[b + i]->d_scratch;
            max_L = std::max(max_L, hs[b + i]->L);
        }
        const hipError_t e = launch_map_steps(a, max_L, stream);
        if (e != hipSuccess) return hip_fail(e, "map-mode launch");
    }
    return LAT_OK;
}

int check_batch(lattice *const *hs, int32_t count)
{
    if (count < 0 || (count > 0 && !hs)) return fail(LAT_EINVAL, "bad batch");
    for (int32_t i = 0; i < count; ++i) {
        if (!live(hs[i])) return fail(LAT_ESTATE, "null or destroyed handle in batch");
        if (hs[i]->L > kMapMaxL) return fail(LAT_EINVAL, "map mode takes lattices with L <= 256");
    }
    std::vector<const lattice *> seen(hs, hs + count);
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
        return fail(LAT_EINVAL, "a lattice appears twice in the batch");
    return LAT_OK;
}

}  // namespace

extern "C" {

int lattice_map_steps(lattice *h, uint64_t first_map, uint32_t n_maps, int32_t partner)
{
    return guarded("lattice_map_steps", [&]() -> int {
        if (!live(h)) return fail(LAT_ESTATE, "null or destroyed handle");
        if (partner != LAT_MAP_ANY && partner != LAT_MAP_NEIGHBOUR) return fail(LAT_EINVAL, "unknown partner rule");
        lattice *one[1] = {h};
        const int rc = check_batch(one, 1);
        if (rc) return rc;
        if (n_maps == 0) return LAT_OK;
        return enqueue_map_steps(one, 1, first_map, n_maps, partner, h->stream);
    });
}

int lattice_map_steps_batch(lattice *const *hs, int32_t count, uint64_t first_map, uint32_t n_maps, int32_t partner,
                            void *hip_stream)
{
    return guarded("lattice_map_steps_batch", [&]() -> int {
        if (partner != LAT_MAP_ANY && partner != LAT_MAP_NEIGHBOUR) return fail(LAT_EINVAL, "unknown partner rule");
        const int rc = check_batch(hs, count);
        if (rc) return rc;
        if (n_maps == 0 || count == 0) return LAT_OK;
        return enqueue_map_steps(hs, count, first_map, n_maps, partner, (hipStream_t)hip_stream);
    });
}

}  // extern "C"
