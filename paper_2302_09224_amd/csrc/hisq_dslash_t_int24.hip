// Dslash instantiations for the triplet GF_FIX32 / SF_INT24 (generated
// shared-exponent format, 24-bit components) / float compute.
#include "hisq_dslash_kernels.h"

namespace hisq {

hipError_t dslash_launch_int24(const DslashArgs &a, int rhs0, const DslashTile &t, hipStream_t st, int *nb) {
    return dsl::launch_tile<GF_FIX32, SF_INT24, float, true>(a, rhs0, t, st, nb);
}

hipError_t dslash_multi_int24(const MultiArgs &m, int long_recon, hipStream_t st) {
    return dsl::launch_multi<GF_FIX32, SF_INT24, float>(m, long_recon, st);
}

}  // namespace hisq
