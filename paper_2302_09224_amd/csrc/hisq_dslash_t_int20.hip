// Dslash instantiation for the triplet GF_FIX16 / SF_INT20 / float compute.
#include "hisq_dslash_kernels.h"

namespace hisq {

hipError_t dslash_launch_int20(const DslashArgs &a, int block, hipStream_t st) {
    return dsl::launch_one<GF_FIX16, SF_INT20, float>(a, block, st);
}

hipError_t dslash_launch_batched_int20(const DslashArgs &a, int block, hipStream_t st) {
    return dsl::launch_batched<GF_FIX16, SF_INT20, float>(a, block, st);
}

}  // namespace hisq
