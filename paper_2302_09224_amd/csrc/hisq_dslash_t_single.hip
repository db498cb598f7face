// Dslash instantiation for the triplet GF_F32 / SF_F32 / float compute.
#include "hisq_dslash_kernels.h"

namespace hisq {

hipError_t dslash_launch_single(const DslashArgs &a, int block, hipStream_t st) {
    return dsl::launch_one<GF_F32, SF_F32, float>(a, block, st);
}

hipError_t dslash_launch_batched_single(const DslashArgs &a, int block, hipStream_t st) {
    return dsl::launch_batched<GF_F32, SF_F32, float>(a, block, st);
}

}  // namespace hisq
