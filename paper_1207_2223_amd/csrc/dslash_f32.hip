// FP32 instantiations of the hopping stencil: FP32 spinors with FP32 or FP16
// 12-real links, FP32 arithmetic.
#include "dslash_impl.h"

namespace wd {

hipError_t dslash_launch_f32(const DslashArgs &a, int lk, int nr, int dag, int epi, int block,
                             int grid, hipStream_t s)
{
    if (lk == LK_F32_12) {
        if (nr == 1) { WD_DSL_DAG(SP_F32, LK_F32_12, 1, SP_F32) }
        if (nr == 2) { WD_DSL_DAG(SP_F32, LK_F32_12, 2, SP_F32) }
        if (nr == 4) { WD_DSL_DAG(SP_F32, LK_F32_12, 4, SP_F32) }
    } else if (lk == LK_F16_12) {
        if (nr == 1) { WD_DSL_DAG(SP_F32, LK_F16_12, 1, SP_F32) }
        if (nr == 2) { WD_DSL_DAG(SP_F32, LK_F16_12, 2, SP_F32) }
        if (nr == 4) { WD_DSL_DAG(SP_F32, LK_F16_12, 4, SP_F32) }
    }
    return hipErrorInvalidValue;
}

}  // namespace wd
