// Dslash instantiation for the triplet GF_FIX32 / SF_INT30 / float compute.
#include "hisq_dslash_kernels.h"

namespace hisq {

hipError_t dslash_launch_int30_fp32(const DslashArgs &a, int block, hipStream_t st) {
    return dsl::launch_one<GF_FIX32, SF_INT30, float>(a, block, st);
}

hipError_t dslash_launch_batched_int30_fp32(const DslashArgs &a, int block, hipStream_t st) {
    (void)a; (void)block; (void)st;
    return hipErrorInvalidValue;  // no batched kernel for this triplet
}

}  // namespace hisq
