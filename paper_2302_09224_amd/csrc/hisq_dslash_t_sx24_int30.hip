// Dslash instantiations for the triplet GF_SX24 (link rows as 24-bit
// shared-exponent records) / SF_INT30 / double compute: the 30-bit spinors of
// the FIX32/INT30 triplet with links of 60 bytes (40 two-row) instead of 72 (48).
#include "hisq_dslash_kernels.h"

namespace hisq {

hipError_t dslash_launch_sx24_int30(const DslashArgs &a, int rhs0, const DslashTile &t, hipStream_t st, int *nb) {
    return dsl::launch_tile<GF_SX24, SF_INT30, double, true>(a, rhs0, t, st, nb);
}

hipError_t dslash_multi_sx24_int30(const MultiArgs &m, int long_recon, hipStream_t st) {
    return dsl::launch_multi<GF_SX24, SF_INT30, double>(m, long_recon, st);
}

}  // namespace hisq
