// Dslash instantiations for the triplet GF_SX24 (link rows as 24-bit
// shared-exponent records) / SF_INT24 / float compute.
#include "hisq_dslash_kernels.h"

namespace hisq {

hipError_t dslash_launch_sx24(const DslashArgs &a, int rhs0, const DslashTile &t, hipStream_t st, int *nb) {
    return dsl::launch_tile<GF_SX24, SF_INT24, float, true>(a, rhs0, t, st, nb);
}

hipError_t dslash_multi_sx24(const MultiArgs &m, int long_recon, hipStream_t st) {
    return dsl::launch_multi<GF_SX24, SF_INT24, float>(m, long_recon, st);
}

}  // namespace hisq
