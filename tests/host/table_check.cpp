// Exhaustive CPU check of the library's host-built tables (test
// infrastructure).  Compiles the library's host source with stub kernel
// launchers, then for every pair state, every choice j and every
// neighbourhood of the two sites (4^8 code combinations):
//   - the transition entry's new state is the j-th configuration of the
//     same-charge set as the oracle lists it (section 3.1), and the delta
//     entry holds the same coefficients with the XOR of old and new codes;
//   - dot4(coef, packed sums) + C lands inside the device table, on an entry
//     whose packed triple is the move's (nD, nV, nJ) computed here from the
//     energy of eq. (3), and whose threshold equals the oracle's threshold.
#include "../../paper_2301_11735_amd/csrc/lattice_api.cpp"

#include <cstdio>

namespace lat {
hipError_t launch_phase_int8(const PhaseArgs &, hipStream_t) { return hipSuccess; }
hipError_t launch_phase_2bit(const PhaseArgs &, const Tuning2Bit &, hipStream_t) { return hipSuccess; }
hipError_t launch_zero_i64(unsigned long long *, int, hipStream_t) { return hipSuccess; }
hipError_t launch_observables(uint8_t *, const void *, int, int, hipStream_t, long long *) { return hipSuccess; }
int words_lanes(int) { return 1; }
hipError_t launch_phase_words(const WordsArgs &, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_advance_words(const WordsArgs &, hipStream_t) { return hipSuccess; }
int words_persistent_capacity(int, int) { return 0; }
hipError_t launch_words_series(const WordsSeriesArgs &, int, hipStream_t) { return hipSuccess; }
hipError_t launch_pack_int8(const int8_t *, uint32_t *, int, hipStream_t) { return hipSuccess; }
hipError_t launch_unpack_int8(const uint32_t *, int8_t *, int, hipStream_t) { return hipSuccess; }
hipError_t launch_sweep_lds(const BatchArgs &, int, int, bool, hipStream_t) { return hipSuccess; }
hipError_t init_kernel_attributes() { return hipSuccess; }
hipError_t init_map_kernel_attributes() { return hipSuccess; }
hipError_t launch_advance(LatDesc *, uint32_t, hipStream_t) { return hipSuccess; }
bool persistent_2bit_supported(int, const Tuning2Bit &, int *, int *) { return false; }
hipError_t launch_sweeps_2bit(const PhaseArgs &, const Tuning2Bit &, uint32_t, unsigned *, unsigned *, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t launch_observables_batch(const BatchArgs &, unsigned long long *, hipStream_t) { return hipSuccess; }
}  // namespace lat

extern "C" uint32_t orc_threshold(double, double, double, double, int, int, int);
extern "C" int orc_pair_config(int, int, int *);

static int dot4(uint32_t a, uint32_t b)
{
    int s = 0;
    for (int k = 0; k < 4; ++k) s += (int)(int8_t)(a >> (8 * k)) * (int)(int8_t)(b >> (8 * k));
    return s;
}

int main()
{
    static const int S[4] = {0, 0, 1, -1}, G[4] = {1, -1, 0, 0};
    const double params[][4] = {{0.25, 0.5, 1.0, 1.2}, {-0.7, 0.3, -1.0, 0.4}, {1e6, 0.5, 1.0, 0.3}};
    long checks = 0;
    for (const auto &pr : params) {
        std::vector<uint32_t> tab, dev, trans, trans_d;
        build_threshold_table(pr[0], pr[1], pr[2], pr[3], tab);
        build_device_table(tab, dev);
        build_transition_table(trans, trans_d);
        for (int nD = -2; nD <= 2; ++nD)
            for (int nV = -16; nV <= 16; ++nV)
                for (int nJ = -16; nJ <= 16; ++nJ)
                    if (threshold_of(tab, nD, nV, nJ) != orc_threshold(pr[0], pr[1], pr[2], pr[3], nD, nV, nJ)) {
                        printf("FAIL threshold (%d,%d,%d)\n", nD, nV, nJ);
                        return 1;
                    }
        for (int st = 0; st < 16; ++st) {
            const int ca = st & 3, cb = st >> 2, q = S[ca] + S[cb];
            const int kq = (q == 2 || q == -2) ? 1 : (q == 0 ? 6 : 4);
            for (int j = 0; j < kq; ++j) {
                const uint32_t coef = trans[2 * (st * 6 + j)], meta = trans[2 * (st * 6 + j) + 1];
                const int ns = (int)(meta >> 16), a1 = ns & 3, b1 = ns >> 2;
                int want[2] = {ca, cb};
                if (kq > 1 && orc_pair_config(q, j, want) != 0) { printf("FAIL set\n"); return 1; }
                if (a1 != want[0] || b1 != want[1]) { printf("FAIL new state st=%d j=%d\n", st, j); return 1; }
                // delta form: same coefficients and offset; every field of the
                // low half holds code_a's change, every field of the high half
                // code_b's
                const uint32_t *d = &trans_d[4 * (st * 6 + j)];
                if (d[0] != coef || d[1] != (meta & 0xFFFFu) || d[3] != 0u) { printf("FAIL delta words st=%d j=%d\n", st, j); return 1; }
                for (int f = 0; f < 16; ++f)
                    if (((d[2] >> (2 * f)) & 3u) != (uint32_t)(f < 8 ? (a1 ^ ca) : (b1 ^ cb))) {
                        printf("FAIL delta field st=%d j=%d f=%d\n", st, j, f);
                        return 1;
                    }
                for (int nb = 0; nb < 65536; ++nb) {
                    int sSa = 0, sGa = 0, sSb = 0, sGb = 0;
                    for (int k = 0; k < 4; ++k) {
                        sSa += S[(nb >> (2 * k)) & 3];
                        sGa += G[(nb >> (2 * k)) & 3];
                        sSb += S[(nb >> (8 + 2 * k)) & 3];
                        sGb += G[(nb >> (8 + 2 * k)) & 3];
                    }
                    const uint32_t bpack = (uint32_t)(sSa + 4) | (uint32_t)(sSb + 4) << 8 |
                                           (uint32_t)(sGa + 4) << 16 | (uint32_t)(sGb + 4) << 24;
                    const int idx = dot4(coef, bpack) + (int)(meta & 0xFFFFu);
                    const int tD = S[a1] * S[a1] + S[b1] * S[b1] - S[ca] * S[ca] - S[cb] * S[cb];
                    const int tV = (S[a1] - S[ca]) * sSa + (S[b1] - S[cb]) * sSb;
                    const int tJ = (G[a1] - G[ca]) * sGa + (G[b1] - G[cb]) * sGb;
                    if (idx < 0 || idx >= kDevTabEntries) { printf("FAIL range st=%d j=%d idx=%d\n", st, j, idx); return 1; }
                    if (dev[2 * idx + 1] != packed_triple(tD, tV, tJ) ||
                        dev[2 * idx] != orc_threshold(pr[0], pr[1], pr[2], pr[3], tD, tV, tJ)) {
                        printf("FAIL entry st=%d j=%d (%d,%d,%d) idx=%d\n", st, j, tD, tV, tJ, idx);
                        return 1;
                    }
                    ++checks;
                }
            }
        }
    }
    printf("OK %ld checks\n", checks);
    return 0;
}
