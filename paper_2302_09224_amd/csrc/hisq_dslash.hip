// hisq_dslash.hip -- dispatch of the Dslash launches on the precision triplet
// gauge/fermion/compute (Sec. 4); the kernels themselves are instantiated in
// hisq_dslash_t_*.hip (one translation unit per triplet).
#include "hisq_internal.h"

namespace hisq {

#define HISQ_DECL_TRIPLET(NAME)                                                           \
    hipError_t dslash_launch_##NAME(const DslashArgs &a, int block, hipStream_t st);       \
    hipError_t dslash_launch_batched_##NAME(const DslashArgs &a, int block, hipStream_t st);
HISQ_DECL_TRIPLET(double)
HISQ_DECL_TRIPLET(single)
HISQ_DECL_TRIPLET(half)
HISQ_DECL_TRIPLET(int20)
HISQ_DECL_TRIPLET(int30)
HISQ_DECL_TRIPLET(int30_fp32)

namespace {
inline int triplet_key(const hisq_fmt &f) { return f.gauge * 100 + f.spinor * 10 + (f.compute == 64 ? 1 : 0); }
}  // namespace

int dslash_blocks(int vh, int block) {
    int nb = (vh + block - 1) / block;
    return (nb + 7) & ~7;
}

int dslash_block_size(const hisq_fmt &, const Geom &, int) { return 256; }

hipError_t launch_dslash(const DslashArgs &a, const hisq_fmt &f, int block, hipStream_t st) {
    switch (triplet_key(f)) {
    case GF_F64 * 100 + SF_F64 * 10 + 1: return dslash_launch_double(a, block, st);
    case GF_F32 * 100 + SF_F32 * 10 + 0: return dslash_launch_single(a, block, st);
    case GF_FIX16 * 100 + SF_HALF16 * 10 + 0: return dslash_launch_half(a, block, st);
    case GF_FIX16 * 100 + SF_INT20 * 10 + 0: return dslash_launch_int20(a, block, st);
    case GF_FIX32 * 100 + SF_INT30 * 10 + 1: return dslash_launch_int30(a, block, st);
    case GF_FIX32 * 100 + SF_INT30 * 10 + 0: return dslash_launch_int30_fp32(a, block, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dslash_batched(const DslashArgs &a, const hisq_fmt &f, int block, hipStream_t st) {
    switch (triplet_key(f)) {
    case GF_F64 * 100 + SF_F64 * 10 + 1: return dslash_launch_batched_double(a, block, st);
    case GF_F32 * 100 + SF_F32 * 10 + 0: return dslash_launch_batched_single(a, block, st);
    case GF_FIX16 * 100 + SF_HALF16 * 10 + 0: return dslash_launch_batched_half(a, block, st);
    case GF_FIX16 * 100 + SF_INT20 * 10 + 0: return dslash_launch_batched_int20(a, block, st);
    case GF_FIX32 * 100 + SF_INT30 * 10 + 1: return dslash_launch_batched_int30(a, block, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hisq
