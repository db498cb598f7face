// Dslash instantiation for the triplet GF_FIX32 / SF_INT30 / double compute.
#include "hisq_dslash_kernels.h"

namespace hisq {

hipError_t dslash_launch_int30(const DslashArgs &a, int block, hipStream_t st) {
    return dsl::launch_one<GF_FIX32, SF_INT30, double>(a, block, st);
}

hipError_t dslash_launch_batched_int30(const DslashArgs &a, int block, hipStream_t st) {
    return dsl::launch_batched<GF_FIX32, SF_INT30, double>(a, block, st);
}

}  // namespace hisq
