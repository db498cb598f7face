// Dslash instantiation for the triplet GF_F64 / SF_F64 / double compute.
#include "hisq_dslash_kernels.h"

namespace hisq {

hipError_t dslash_launch_double(const DslashArgs &a, int block, hipStream_t st) {
    return dsl::launch_one<GF_F64, SF_F64, double>(a, block, st);
}

hipError_t dslash_launch_batched_double(const DslashArgs &a, int block, hipStream_t st) {
    return dsl::launch_batched<GF_F64, SF_F64, double>(a, block, st);
}

}  // namespace hisq
