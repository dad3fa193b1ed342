// Stencil instantiations of the t-walking kernel (t neighbours in registers):
// FP16 spinors (per-site FP32 norm) with FP32 or FP16 12-real links, adjoint hopping.
#include "dslash_impl.h"

namespace wd {

hipError_t dslash_tw_launch_f16_d1(const DslashArgs &a, int lk, int nr, int epi, int block, int grid,
                                  hipStream_t s)
{
    if (lk == LK_F32_12) {
        WD_DSL_TW_SHAPE(SP_F16, LK_F32_12, 1, true)
        WD_DSL_TW_SHAPE(SP_F16, LK_F32_12, 2, true)
        WD_DSL_TW_SHAPE(SP_F16, LK_F32_12, 3, true)
    }
    if (lk == LK_F16_12) {
        WD_DSL_TW_SHAPE(SP_F16, LK_F16_12, 1, true)
        WD_DSL_TW_SHAPE(SP_F16, LK_F16_12, 2, true)
        WD_DSL_TW_SHAPE(SP_F16, LK_F16_12, 3, true)
    }
    return hipErrorInvalidValue;
}

}  // namespace wd
