// Dslash instantiations for the triplet GF_F64 / SF_F64 / double compute.
#include "hisq_dslash_kernels.h"

namespace hisq {

hipError_t dslash_launch_double(const DslashArgs &a, int rhs0, const DslashTile &t, hipStream_t st, int *nb) {
    return dsl::launch_tile<GF_F64, SF_F64, double, true>(a, rhs0, t, st, nb);
}

hipError_t dslash_multi_double(const MultiArgs &m, int long_recon, hipStream_t st) {
    return dsl::launch_multi<GF_F64, SF_F64, double>(m, long_recon, st);
}

}  // namespace hisq
