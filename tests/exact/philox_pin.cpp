// Host-side call into rocRAND's Philox4x32-10 bijection, used as an
// independent library implementation to pin the oracle's Philox.
// Test infrastructure; compiled with g++ against the rocRAND headers.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

namespace {
struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 bijection(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
}  // namespace

extern "C" void pin_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int n)
{
    Engine e;
    for (int i = 0; i < n; ++i) {
        uint4 c{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
        uint2 k{key[2 * i], key[2 * i + 1]};
        uint4 r = e.bijection(c, k);
        out[4 * i] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
    }
}
