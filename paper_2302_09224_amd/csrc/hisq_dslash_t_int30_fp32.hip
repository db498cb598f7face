// Dslash instantiations for the triplet GF_FIX32 / SF_INT30 / float compute.
#include "hisq_dslash_kernels.h"

namespace hisq {

hipError_t dslash_launch_int30_fp32(const DslashArgs &a, int rhs0, const DslashTile &t, hipStream_t st, int *nb) {
    return dsl::launch_tile<GF_FIX32, SF_INT30, float, false>(a, rhs0, t, st, nb);
}

hipError_t dslash_multi_int30_fp32(const MultiArgs &m, int long_recon, hipStream_t st) {
    return dsl::launch_multi<GF_FIX32, SF_INT30, float>(m, long_recon, st);
}

}  // namespace hisq
